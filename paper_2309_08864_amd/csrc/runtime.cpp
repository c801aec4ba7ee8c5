// runtime.cpp -- the executor: runs a plan's schedule on HIP streams.
//
// Streams (Algorithm 1 spreads chunks over streams so that copy-in, kernels
// and copy-out of different chunks overlap, Sec. IV-A and Sec. III).  On
// MI355X the host link is the scarce resource and each direction has its own
// DMA engine, so the executor gives each direction one in-order stream:
//   streams[0]        copy-in (host -> HBM), one chunk after another;
//   streams[1]        copy-out (HBM -> host), one chunk after another;
//   streams[2..n-1]   compute: region-sharing copies and fused kernels,
//                     chunk g on compute stream g mod (n - 2).
// With fewer streams the roles share: n = 2 puts compute on the copy-in
// stream, n = 1 runs everything in order on one stream.  Two copies never
// split one direction's bandwidth, and kernels of consecutive chunks may
// overlap each other when there are several compute streams (Sec. V-D).
// Dependencies are HIP events:
//   * copy-in of chunk g waits copy-out of chunk g - n_slots (slot reuse);
//   * compute of g waits its copy-in; copy-out of g waits its compute;
//   * region sharing: every access to a slot of the sharing buffer waits
//     for the previous access to that slot, so chunk i reads what chunk i-1
//     wrote before chunk i overwrites it (read, then write, as Algorithm 1
//     says; per step for the comparison method);
//   * host array, in place across rounds: round t+1's copy-in of chunk i
//     waits round t's copy-out of chunks i and i+1, which write the planes it
//     reads.  Within a round, chunk i's copy-out (which overwrites r k'
//     planes below its own range) follows chunk i-1's copy-in through the
//     region-sharing chain.
// Nothing synchronises the device between rounds.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <string>

#include "launch.hpp"
#include "aux.hpp"
#include "plan.hpp"

namespace so2dr {

Plan::~Plan() {
  for (auto e : ev_op) hipEventDestroy(e);
  for (auto e : ev_rs) hipEventDestroy(e);
  for (auto e : ev_d2h) hipEventDestroy(e);
  for (auto e : ev_h2d) hipEventDestroy(e);
  for (auto e : ev_comp) hipEventDestroy(e);
  for (auto e : ev_t) hipEventDestroy(e);
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                   \
      return SO2DR_E_HIP;                                                             \
    }                                                                                 \
  } while (0)

static int ensure_events(std::vector<hipEvent_t> &v, size_t n, unsigned flags) {
  while (v.size() < n) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, flags));
    v.push_back(e);
  }
  return SO2DR_OK;
}

void drain_streams(Plan &P) {
  for (hipStream_t s : P.streams) (void)hipStreamSynchronize(s);
  (void)hipGetLastError();
}

int check_pinned(const void *p, size_t bytes, const char *what) {
  if (!p) {
    set_error(std::string(what) + " is null");
    return SO2DR_E_INVALID;
  }
  const char *c = static_cast<const char *>(p);
  for (const char *q : {c, c + (bytes ? bytes - 1 : 0)}) {
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    hipError_t e = hipPointerGetAttributes(&a, q);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error(std::string(what) + " is not pinned host memory");
      return SO2DR_E_NOT_PINNED;
    }
    if (a.type != hipMemoryTypeHost) {
      set_error(std::string(what) + " is not pinned host memory");
      return SO2DR_E_NOT_PINNED;
    }
  }
  return SO2DR_OK;
}

char *mapped_host(const void *p, size_t bytes) {
  if (!p || bytes == 0) return nullptr;
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, p) != hipSuccess || a.type != hipMemoryTypeHost || !a.devicePointer) {
    (void)hipGetLastError();
    return nullptr;
  }
  void *base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, a.devicePointer) != hipSuccess || !base) {
    (void)hipGetLastError();
    return nullptr;
  }
  // the whole range must lie inside the one allocation that holds p
  const uintptr_t d = (uintptr_t)a.devicePointer, b = (uintptr_t)base;
  if (d < b || d - b > size || size - (d - b) < bytes) return nullptr;
  return static_cast<char *>(a.devicePointer);
}

static bool kernel_copyable(const void *x, const void *y, size_t n) {
  return (((uintptr_t)x | (uintptr_t)y | (uintptr_t)n) & 15) == 0;
}

int copy_to_device(void *dst, const void *src_host, size_t n, const void *host_base, char *dev_base,
                   hipStream_t s) {
  if (n == 0) return SO2DR_OK;
  if (dev_base) {
    const char *src = dev_base + (static_cast<const char *>(src_host) - static_cast<const char *>(host_base));
    if (kernel_copyable(dst, src, n)) {
      if (launch_dcopy(dst, src, n, s, kHostCopyWgs)) {
        set_error("host copy kernel launch failed");
        return SO2DR_E_HIP;
      }
      return SO2DR_OK;
    }
  }
  HIPCHK(hipMemcpyAsync(dst, src_host, n, hipMemcpyHostToDevice, s));
  return SO2DR_OK;
}

int copy_to_host(void *dst_host, const void *src, size_t n, const void *host_base, char *dev_base,
                 hipStream_t s) {
  if (n == 0) return SO2DR_OK;
  if (dev_base) {
    char *dst = dev_base + (static_cast<char *>(dst_host) - static_cast<const char *>(host_base));
    if (kernel_copyable(dst, src, n)) {
      if (launch_dcopy(dst, src, n, s, kHostCopyWgs)) {
        set_error("host copy kernel launch failed");
        return SO2DR_E_HIP;
      }
      return SO2DR_OK;
    }
  }
  HIPCHK(hipMemcpyAsync(dst_host, src, n, hipMemcpyDeviceToHost, s));
  return SO2DR_OK;
}

int bind_plan(Plan &P, void *arena, size_t bytes, void *const *streams, int n_streams) {
  if (!arena || (reinterpret_cast<uintptr_t>(arena) & 255)) {
    set_error("arena must be a non-null 256-byte aligned device pointer");
    return SO2DR_E_INVALID;
  }
  if (bytes < P.workspace) {
    set_error("arena smaller than the plan's workspace");
    return SO2DR_E_INVALID;
  }
  if (!streams || n_streams < 1) {
    set_error("at least one stream is needed");
    return SO2DR_E_INVALID;
  }
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, arena) != hipSuccess || a.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    set_error("arena is not device memory");
    return SO2DR_E_INVALID;
  }
  P.arena = static_cast<char *>(arena);
  P.arena_bytes = bytes;
  P.streams.clear();
  for (int i = 0; i < n_streams; ++i) P.streams.push_back(static_cast<hipStream_t>(streams[i]));
  P.bound = true;
  return SO2DR_OK;
}

void schedule_deps(const Plan &P, const std::vector<so2dr_op> &ops, int ns, std::vector<int> *stream,
                   std::vector<int64_t> *waits) {
  const size_t n = ops.size();
  stream->assign(n, 0);
  waits->assign(n * kMaxWaits, -1);
  const int nc = ns >= 3 ? ns - 2 : 1;
  int64_t n_seq = 0;
  for (const so2dr_op &op : ops) n_seq = std::max<int64_t>(n_seq, (int64_t)op.round * P.d + op.chunk + 1);
  std::vector<int64_t> h2d_of(n_seq, -1), d2h_of(n_seq, -1);
  std::map<int64_t, int64_t> last_rs;   // region-sharing slot -> its last access
  int64_t comp_g = -1;
  for (size_t k = 0; k < n; ++k) {
    const so2dr_op &op = ops[k];
    const int64_t g = (int64_t)op.round * P.d + op.chunk;
    int64_t *w = waits->data() + k * kMaxWaits;
    int nw = 0;
    switch (op.kind) {
      case SO2DR_OP_H2D:
        (*stream)[k] = 0;
        // slot reuse: the copy-out of the chunk that held this slot before
        if (g >= P.n_slots) w[nw++] = d2h_of[g - P.n_slots];
        // host array in place: last round's copy-outs of chunks i and i+1
        // write the planes this copy-in reads
        if (op.round > 0) {
          w[nw++] = d2h_of[g - P.d];
          if (op.chunk + 1 < P.d) w[nw++] = d2h_of[g - P.d + 1];
        }
        h2d_of[g] = (int64_t)k;
        break;
      case SO2DR_OP_RS_READ:
      case SO2DR_OP_RS_WRITE:
      case SO2DR_OP_KERNEL: {
        (*stream)[k] = ns >= 3 ? 2 + (int)(g % nc) : 0;
        if (comp_g != g) {   // first compute op of the chunk: its input is in HBM
          w[nw++] = h2d_of[g];
          comp_g = g;
        }
        if (op.kind != SO2DR_OP_KERNEL) {   // read, then write, in schedule order
          auto it = last_rs.find(op.pool_off);
          if (it != last_rs.end()) w[nw++] = it->second;
          last_rs[op.pool_off] = (int64_t)k;
        }
        break;
      }
      case SO2DR_OP_D2H:
        (*stream)[k] = ns >= 2 ? 1 : 0;
        w[nw++] = (int64_t)k - 1;   // the chunk's last compute op
        d2h_of[g] = (int64_t)k;
        break;
      default:
        break;
    }
    // drop waits on ops of the same stream (list order covers them) and on
    // nothing (-1), and duplicates
    int m = 0;
    for (int i = 0; i < nw; ++i) {
      const int64_t x = w[i];
      bool keep = x >= 0 && (*stream)[x] != (*stream)[k];
      for (int j = 0; j < m && keep; ++j) keep = w[j] != x;
      if (keep) w[m++] = x;
    }
    for (int i = m; i < kMaxWaits; ++i) w[i] = -1;
  }
}

// Run `steps` steps from host_in into host_out (may alias).
int execute(Plan &P, const void *host_in, void *host_out, int steps, so2dr_stats *st) {
  if (!P.bound) {
    set_error("plan is not bound to device memory and streams");
    return SO2DR_E_UNBOUND;
  }
  if (steps < 0 || steps > P.T) {
    set_error("steps must be in [0, T]");
    return SO2DR_E_INVALID;
  }
  const size_t field = (size_t)P.N * P.plane_bytes();
  int rc = check_pinned(host_in, field, "input host array");
  if (rc) return rc;
  rc = check_pinned(host_out, field, "output host array");
  if (rc) return rc;
  // device mappings for copy kernels (null: hipMemcpyAsync)
  char *dev_in = nullptr, *dev_out = nullptr;
  bool k_in = P.copy_engine == SO2DR_COPY_KERNEL;
  if (k_in || P.copy_engine == SO2DR_COPY_KERNEL_OUT) {
    dev_in = mapped_host(host_in, field);
    dev_out = host_out == host_in ? dev_in : mapped_host(host_out, field);
    if (!dev_in || !dev_out) {
      if (P.copy_engine_forced) {
        set_error("copy kernels need each host array inside one page-locked allocation mapped into the device");
        return SO2DR_E_NOT_PINNED;
      }
      dev_in = dev_out = nullptr;
      k_in = false;
    }
  }
  so2dr_stats S;
  std::memset(&S, 0, sizeof(S));
  const auto t_start = std::chrono::steady_clock::now();
  if (steps == 0) {
    if (host_in != host_out) std::memcpy(host_out, host_in, field);
    if (st) *st = S;
    return SO2DR_OK;
  }
  int64_t computed = 0;
  const std::vector<so2dr_op> ops = build_ops(P, steps, &computed);
  const int ns = (int)P.streams.size();
  std::vector<int> strm;
  std::vector<int64_t> waits;
  schedule_deps(P, ops, ns, &strm, &waits);
  // an event after every op that a later op on another stream waits for
  std::vector<char> awaited(ops.size(), 0);
  for (int64_t x : waits)
    if (x >= 0) awaited[(size_t)x] = 1;
  rc = ensure_events(P.ev_op, ops.size(), hipEventDisableTiming);
  if (rc) return rc;
  if (P.timing) {
    rc = ensure_events(P.ev_t, 2 * ops.size(), hipEventDefault);
    if (rc) return rc;
  }
  const size_t pb = P.plane_bytes();
  const char *hin = static_cast<const char *>(host_in);
  char *hout = static_cast<char *>(host_out);
  std::string msg;
  // every operation is enqueued here; on a failure part-way, the work
  // already queued is drained before returning (so the caller may release
  // the arena at once)
  const int64_t fail_at = P.fail_after_ops;
  P.fail_after_ops = -1;   // one run only
  auto enqueue = [&]() -> int {
  for (size_t k = 0; k < ops.size(); ++k) {
    const so2dr_op &op = ops[k];
    hipStream_t s = P.streams[strm[k]];
    if ((int64_t)k == fail_at) {
      set_error("injected failure after " + std::to_string(k) + " operations (so2dr_plan_set_fail_after)");
      return SO2DR_E_HIP;
    }
    // cross-stream waits, enqueued before the op's timing start
    for (int i = 0; i < kMaxWaits; ++i) {
      const int64_t x = waits[k * kMaxWaits + i];
      if (x >= 0) HIPCHK(hipStreamWaitEvent(s, P.ev_op[(size_t)x], 0));
    }
    if (P.timing) HIPCHK(hipEventRecord(P.ev_t[2 * k], s));
    switch (op.kind) {
      case SO2DR_OP_H2D: {
        const char *base = op.round == 0 ? hin : hout;
        char *dev = !k_in ? nullptr : op.round == 0 ? dev_in : dev_out;
        char *dst = P.slot_buf(op.slot, op.buf_out) + (size_t)(op.z0 - op.buf_z0) * pb;
        rc = copy_to_device(dst, base + (size_t)op.z0 * pb, (size_t)(op.z1 - op.z0) * pb, base, dev, s);
        if (rc) return rc;
        S.bytes_h2d += (uint64_t)(op.z1 - op.z0) * pb;
        break;
      }
      case SO2DR_OP_RS_READ:
      case SO2DR_OP_RS_WRITE: {
        const size_t n = (size_t)(op.z1 - op.z0) * pb;
        char *pool = P.rs_pool() + (size_t)op.pool_off * pb;
        // a copy kernel on the compute stream, not the runtime's copy path,
        // which may hand device copies to a DMA engine the host copies use
        int crc;
        if (op.kind == SO2DR_OP_RS_READ) {
          char *dst = P.slot_buf(op.slot, op.buf_out) + (size_t)(op.z0 - op.buf_z0) * pb;
          crc = launch_dcopy(dst, pool, n, s);
        } else {
          const char *src = P.slot_buf(op.slot, op.buf_in) + (size_t)(op.z0 - op.buf_z0) * pb;
          crc = launch_dcopy(pool, src, n, s);
        }
        if (crc) {
          set_error("region-sharing copy kernel launch failed");
          return SO2DR_E_HIP;
        }
        S.bytes_d2d += n;
        break;
      }
      case SO2DR_OP_KERNEL: {
        LaunchParams lp;
        lp.stencil = P.stencil;
        lp.kl = op.levels;
        lp.in = P.slot_buf(op.slot, op.buf_in);
        lp.out = P.slot_buf(op.slot, op.buf_out);
        lp.buf_z0 = op.buf_z0;
        lp.out_z0 = op.out_z0;
        lp.plane = P.plane;
        lp.nx = (int)P.NX;
        lp.ny = (int)P.NY;
        lp.per_x = P.per_x;
        lp.per_y = P.per_y;
        lp.n_axis = P.N;
        lp.in_lo = op.in_z0;
        lp.in_hi = op.in_z1;
        lp.out_lo = op.z0;
        lp.out_hi = op.z1;
        lp.weights = P.weights.data();
        lp.npts = (int)P.weights.size();
        lp.ras = P.ras;
        rc = launch_tb(P.dtype, lp, s, &msg);
        if (rc) {
          set_error(msg);
          return rc;
        }
        const uint64_t alg = (uint64_t)((op.in_z1 - op.in_z0) + (op.z1 - op.z0)) * pb;
        S.kernel_launches += 1;
        S.kernel_alg_bytes += alg;
        if (op.levels >= 1 && op.levels <= 8) {
          S.launches_by_levels[op.levels - 1] += 1;
          S.alg_bytes_by_levels[op.levels - 1] += alg;
        }
        break;
      }
      case SO2DR_OP_D2H: {
        const char *src = P.slot_buf(op.slot, op.buf_in) + (size_t)(op.z0 - op.buf_z0) * pb;
        rc = copy_to_host(hout + (size_t)op.z0 * pb, src, (size_t)(op.z1 - op.z0) * pb, hout, dev_out, s);
        if (rc) return rc;
        S.bytes_d2h += (uint64_t)(op.z1 - op.z0) * pb;
        if (op.chunk == P.d - 1) S.rounds_done = op.round + 1;
        break;
      }
      default:
        set_error("corrupt schedule");
        return SO2DR_E_INVALID;
    }
    if (P.timing) HIPCHK(hipEventRecord(P.ev_t[2 * k + 1], s));
    if (awaited[k]) HIPCHK(hipEventRecord(P.ev_op[k], s));
  }
  return SO2DR_OK;
  };
  rc = enqueue();
  if (rc) {
    // what was queued has finished: rounds_done counts the rounds whose
    // copy-out of the last chunk was queued
    drain_streams(P);
    S.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (st) *st = S;
    return rc;
  }
  for (hipStream_t s : P.streams) HIPCHK(hipStreamSynchronize(s));
  const auto t_end = std::chrono::steady_clock::now();
  S.wall_ms = std::chrono::duration<double, std::milli>(t_end - t_start).count();
  S.cell_updates = (uint64_t)P.N * (uint64_t)P.plane * (uint64_t)steps;
  S.cell_updates_done = (uint64_t)computed * (uint64_t)P.plane;
  if (P.timing) {
    for (size_t k = 0; k < ops.size(); ++k) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, P.ev_t[2 * k], P.ev_t[2 * k + 1]));
      switch (ops[k].kind) {
        case SO2DR_OP_H2D: S.h2d_ms += ms; break;
        case SO2DR_OP_D2H: S.d2h_ms += ms; break;
        case SO2DR_OP_KERNEL:
          S.kernel_ms += ms;
          if (ops[k].levels >= 1 && ops[k].levels <= 8) S.kernel_ms_by_levels[ops[k].levels - 1] += ms;
          break;
        default: S.d2d_ms += ms; break;
      }
    }
  }
  if (st) *st = S;
  return SO2DR_OK;
}

int kernel_bench(const Plan &P, int levels, void *dev_in, void *dev_out, int64_t in_planes, int reps,
                 hipStream_t s, double *ms) {
  if (!dev_in || !dev_out || !ms || reps < 1 || levels < 0 || levels > P.max_k_on) {
    set_error("null buffer or output, reps < 1, or levels outside [0, max_k_on]");
    return SO2DR_E_INVALID;
  }
  const int64_t halo = (int64_t)levels * P.r;
  if (in_planes <= 2 * halo || in_planes > P.N) {
    set_error("in_planes must exceed 2 * levels * radius and not exceed the cut axis");
    return SO2DR_E_INVALID;
  }
  const size_t pb = P.plane_bytes();
  // the planes sit in the middle of the cut axis: an interior chunk
  const int64_t base = (P.N - in_planes) / 2;
  LaunchParams lp;
  lp.stencil = P.stencil;
  lp.kl = levels;
  lp.in = dev_in;
  lp.out = dev_out;
  lp.buf_z0 = base;
  lp.out_z0 = base;
  lp.plane = P.plane;
  lp.nx = (int)P.NX;
  lp.ny = (int)P.NY;
  lp.per_x = P.per_x;
  lp.per_y = P.per_y;
  lp.n_axis = P.N;
  lp.in_lo = base;
  lp.in_hi = base + in_planes;
  lp.out_lo = base + halo;
  lp.out_hi = base + in_planes - halo;
  lp.weights = P.weights.data();
  lp.npts = (int)P.weights.size();
  lp.ras = P.ras;
  std::string msg;
  auto launch = [&]() -> int {
    if (levels == 0) {
      if (launch_dcopy(dev_out, dev_in, (size_t)in_planes * pb, s)) {
        set_error("copy kernel launch failed");
        return SO2DR_E_HIP;
      }
      return SO2DR_OK;
    }
    const int rc = launch_tb(P.dtype, lp, s, &msg);
    if (rc) set_error(msg);
    return rc;
  };
  int rc = launch();   // first launch: one-time set-up outside the timing
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    set_error("hipEventCreate failed");
    return SO2DR_E_HIP;
  }
  hipError_t e = hipEventRecord(e0, s);
  for (int i = 0; i < reps && e == hipSuccess && rc == SO2DR_OK; ++i) rc = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess && rc == SO2DR_OK) e = hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc || e != hipSuccess) (void)hipStreamSynchronize(s);  // the caller may free the buffers next
  if (rc) return rc;
  if (e != hipSuccess) {
    set_error(std::string("kernel timing: ") + hipGetErrorString(e));
    return SO2DR_E_HIP;
  }
  *ms = (double)t / reps;
  return SO2DR_OK;
}

int link_probe(void *host_a, void *host_b, void *dev_a, void *dev_b, size_t bytes, int pieces,
               hipStream_t s_in, hipStream_t s_out, int reps, double *gbps) {
  if (!host_a || !host_b || !dev_a || !dev_b || !gbps || bytes == 0 || reps < 1 || s_in == s_out ||
      pieces < 1 || bytes % (size_t)pieces) {
    set_error("null buffer or output, zero bytes, reps < 1, one stream for both directions, or bytes "
              "not a multiple of pieces");
    return SO2DR_E_INVALID;
  }
  const size_t piece = bytes / (size_t)pieces;
  int rc = check_pinned(host_a, bytes, "host_a");
  if (rc) return rc;
  rc = check_pinned(host_b, bytes, "host_b");
  if (rc) return rc;
  // mode 0: host -> HBM alone; 1: HBM -> host alone; 2: both at once.  On
  // an error the copies already queued are drained before returning: the
  // caller may free the buffers as soon as the call fails.
  auto passes = [&]() -> int {
    for (int mode = 0; mode < 3; ++mode) {
      double best = 0.0;
      for (int rep = 0; rep <= reps; ++rep) {   // the first pass warms up
        HIPCHK(hipStreamSynchronize(s_in));
        HIPCHK(hipStreamSynchronize(s_out));
        const auto t0 = std::chrono::steady_clock::now();
        // the pieces of both directions are queued interleaved, as the
        // executor queues one chunk's copy-in and an earlier chunk's copy-out
        for (int k = 0; k < pieces; ++k) {
          const size_t off = (size_t)k * piece;
          if (mode != 1)
            HIPCHK(hipMemcpyAsync(static_cast<char *>(dev_a) + off, static_cast<char *>(host_a) + off, piece,
                                  hipMemcpyHostToDevice, s_in));
          if (mode != 0)
            HIPCHK(hipMemcpyAsync(static_cast<char *>(host_b) + off, static_cast<char *>(dev_b) + off, piece,
                                  hipMemcpyDeviceToHost, s_out));
        }
        HIPCHK(hipStreamSynchronize(s_in));
        HIPCHK(hipStreamSynchronize(s_out));
        const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        const double rate = (mode == 2 ? 2.0 : 1.0) * (double)bytes / sec / 1e9;
        if (rep > 0 && rate > best) best = rate;
      }
      gbps[mode] = best;
    }
    return SO2DR_OK;
  };
  rc = passes();
  if (rc != SO2DR_OK) {
    (void)hipStreamSynchronize(s_in);
    (void)hipStreamSynchronize(s_out);
  }
  return rc;
}

int launch_tb(int dtype, const LaunchParams &p, hipStream_t stream, std::string *msg) {
  switch (dtype) {
    case SO2DR_F32: return launch_tb_f32(p, stream, msg);
    case SO2DR_F64: return launch_tb_f64(p, stream, msg);
    case SO2DR_BF16: return launch_tb_bf16(p, stream, msg);
    case SO2DR_F16: return launch_tb_f16(p, stream, msg);
    default:
      if (msg) *msg = "unknown storage type";
      return SO2DR_E_INVALID;
  }
}

}  // namespace so2dr
