// plan.hpp -- host-side plan: geometry, schedule and bound device state.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/so2dr.h"

namespace so2dr {

void set_error(const std::string &msg);

struct Plan {
  // ---- problem (validated copy of the descriptor)
  int ndim = 0, shape = 0, r = 0, dtype = 0, stencil = -1;
  int64_t nx = 0, ny = 0, nz = 0;
  int64_t NX = 0, NY = 0, N = 0;   // in-plane extents and cut-axis length
  int64_t plane = 0;               // elements per plane
  size_t elem = 0;                 // bytes per stored element
  int per_x = 0, per_y = 0;        // periodic flags of the in-plane axes
  std::vector<double> weights;     // lexicographic
  // ---- plan
  int T = 0, K = 0, k_on = 0, d = 0, n_slots = 0, max_k_on = 0;
  std::vector<int64_t> bnd;        // chunk i owns planes [bnd[i], bnd[i+1])
  int64_t slot_planes = 0;
  size_t buf_bytes = 0;            // one ping-pong buffer (256-aligned)
  size_t rs_bytes = 0, scratch_bytes = 0, workspace = 0, budget = 0;
  bool adjoint = false;
  int bufs_per_slot = 2;           // 2 ping-pong buffers (1 in a lean plan)
  int shared_bufs = 0;             // adjoint: working buffers the compute stream shares
  bool resreu = false;             // comparison method: per-step sharing, single-step kernels
  int ras = 0;                     // 16-bit storage rounded only where a launch stores
  int copy_engine = SO2DR_COPY_DMA;  // host copies: DMA engines or copy kernels
  bool copy_engine_forced = false;   // chosen by the caller, not automatically
  bool lean = false;               // 1 buffer per slot, kernels split into shifted sub-blocks
  int lean_block = 0;              // output planes per sub-block launch
  int64_t lean_extra = 0;          // spare planes below the round-start data
  // ---- bound state
  char *arena = nullptr;
  size_t arena_bytes = 0;
  std::vector<hipStream_t> streams;
  bool bound = false;
  bool timing = false;
  int64_t fail_after_ops = -1;     // testing aid: the next run fails after this many ops
  std::vector<hipEvent_t> ev_rs, ev_d2h, ev_h2d, ev_comp;   // adjoint sweep: round * d + chunk
  std::vector<hipEvent_t> ev_op;           // forward runs: completion of op k (when awaited)
  std::vector<hipEvent_t> ev_t;            // timing pairs, 2 per op
  ~Plan();

  size_t plane_bytes() const { return (size_t)plane * elem; }
  // buffer `which` of a slot; indices from bufs_per_slot on name the shared
  // working buffers, the same for every slot
  char *slot_buf(int slot, int which) const {
    if (which >= bufs_per_slot)
      return arena + ((size_t)n_slots * bufs_per_slot + (size_t)(which - bufs_per_slot)) * buf_bytes;
    return arena + ((size_t)slot * bufs_per_slot + (size_t)which) * buf_bytes;
  }
  char *rs_pool(int which = 0) const {
    return arena + ((size_t)n_slots * bufs_per_slot + (size_t)shared_bufs) * buf_bytes +
           (size_t)which * rs_bytes;
  }
  int n_rs() const { return adjoint ? 2 : 1; }
  char *scratch() const { return rs_pool(0) + (size_t)n_rs() * rs_bytes; }
};

// Geometry of round `t` for a run of `steps` steps.
int round_depth(const Plan &P, int steps, int t);
int n_rounds_for(const Plan &P, int steps);
// Valid planes of chunk i at level s of a round of depth kp (Sec. IV-B).
int64_t area_lo(const Plan &P, int i, int kp, int s);
int64_t area_hi(const Plan &P, int i, int kp, int s);

// The executor's dependency rules for a schedule run on n_streams streams:
// the stream index of every op and the (at most kMaxWaits) earlier ops whose
// completion it waits for, -1 padded.  Ops on one stream run in list order.
constexpr int kMaxWaits = SO2DR_MAX_WAITS;
void schedule_deps(const Plan &P, const std::vector<so2dr_op> &ops, int n_streams,
                   std::vector<int> *stream, std::vector<int64_t> *waits);

// Build the schedule for `steps` steps (Algorithm 1 unrolled).  Also returns
// the number of cell-plane updates computed (including redundant ones).
std::vector<so2dr_op> build_ops(const Plan &P, int steps, int64_t *planes_computed);

// Validate and plan; returns 0 or a negative code with set_error().
int make_plan(const so2dr_desc &d, Plan *out);

size_t dtype_size(int dtype);
int stencil_id(int ndim, int shape, int r);
int expected_points(int ndim, int shape, int r);

// Automatic copy engine: copy kernels when the largest chunk copy is below
// kKernelCopyBelow bytes and a run queues more than kKernelCopyQueued host
// copies at once; the DMA engines otherwise.
constexpr size_t kKernelCopyBelow = (size_t)512 << 20;
constexpr int64_t kKernelCopyQueued = 256;
// Workgroups of one host-copy kernel (about the link's rate per direction).
constexpr int kHostCopyWgs = 64;

// Wait for whatever a failed run already queued on the plan's streams
// (errors ignored; the caller reports the first one).
void drain_streams(Plan &P);

// Device address of the host range [p, p + bytes) when it lies inside one
// page-locked allocation mapped into the current device, else null.
char *mapped_host(const void *p, size_t bytes);
// One host <-> HBM copy of n bytes on stream s.  With dev_base (the device
// address of host_base from mapped_host) a copy kernel moves the bytes
// through the mapping; without, hipMemcpyAsync.  Returns 0 or SO2DR_E_HIP.
int copy_to_device(void *dst, const void *src_host, size_t n, const void *host_base, char *dev_base,
                   hipStream_t s);
int copy_to_host(void *dst_host, const void *src, size_t n, const void *host_base, char *dev_base,
                 hipStream_t s);

}  // namespace so2dr
