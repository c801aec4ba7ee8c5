// planner.cpp -- the chunk planner: pure host code, no device calls.
//
// Geometry (paper Algorithm 1 and Sec. IV):
//   * the cut axis [0, N) is split into d chunks [b_{i-1}, b_i);
//   * rounds of K steps (K = tb_depth, the paper's S_TB / k_off); the last
//     round runs the remainder T - (N_t - 1) K  (Algorithm 1, first lines);
//   * chunk i receives its own planes from the host and the 2 r k' planes
//     below them at round-start level from the region-sharing buffer, which
//     chunk i-1 filled with its top 2 r k' planes (read first, then write,
//     as Algorithm 1 orders it);
//   * at level s of the round its valid area is
//       lo_s = b_{i-1} - 2 r k' + s r   (0 for the first chunk)
//       hi_s = b_i - s r                (N for the last chunk),
//     the parallelogram of Sec. IV-B / Sec. VI: the overlap with chunk i-1
//     is recomputed redundantly so that kernels can fuse steps;
//   * the output [b_{i-1} - r k', b_i - r k') of all chunks partitions [0, N);
//   * per round, floor(k'/k_on) launches of k_on fused steps plus one launch
//     of k' mod k_on steps when that is non-zero (Algorithm 1 inner loop).
// Memory (Sec. III constraint, counted honestly): n_slots slots of two
// ping-pong buffers each, sized for the largest chunk plus its 2 r K halo,
// plus the region-sharing buffer of 2 r K planes, must fit the budget.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "aux.hpp"
#include "depths.hpp"
#include "plan.hpp"
#include "rates.hpp"

namespace so2dr {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t dtype_size(int dtype) {
  switch (dtype) {
    case SO2DR_F32: return 4;
    case SO2DR_F64: return 8;
    case SO2DR_BF16: return 2;
    case SO2DR_F16: return 2;
    default: return 0;
  }
}

int stencil_id(int ndim, int shape, int r) {
  if (ndim == 2 && shape == SO2DR_STAR && r == 1) return ST_2D_STAR_R1;
  if (ndim == 2 && shape == SO2DR_BOX && r >= 1 && r <= 4) return ST_2D_BOX_R1 + (r - 1);
  if (ndim == 3 && shape == SO2DR_STAR && r == 1) return ST_3D_STAR_R1;
  if (ndim == 3 && shape == SO2DR_STAR && r == 2) return ST_3D_STAR_R2;
  if (ndim == 3 && shape == SO2DR_BOX && r == 1) return ST_3D_BOX_R1;
  return -1;
}

int expected_points(int ndim, int shape, int r) {
  const int w = 2 * r + 1;
  if (shape == SO2DR_BOX) return ndim == 2 ? w * w : w * w * w;
  return 1 + 2 * ndim * r;
}

int max_depth(int dtype, int stencil) {
  if (dtype < 0 || dtype > 3 || stencil < 0 || stencil >= ST_COUNT) return 0;
  return kMaxDepth[dtype][stencil];
}

int n_rounds_for(const Plan &P, int steps) { return steps <= 0 ? 0 : (steps + P.K - 1) / P.K; }

int round_depth(const Plan &P, int steps, int t) {
  const int nt = n_rounds_for(P, steps);
  if (t == nt - 1 && steps % P.K != 0) return steps % P.K;
  return P.K;
}

int64_t area_lo(const Plan &P, int i, int kp, int s) {
  if (i == 0) return 0;
  if (P.resreu) return P.bnd[i] - (int64_t)s * P.r;  // no redundant overlap
  return P.bnd[i] - 2 * (int64_t)P.r * kp + (int64_t)s * P.r;
}

int64_t area_hi(const Plan &P, int i, int kp, int s) {
  if (i == P.d - 1) return P.N;
  return P.bnd[i + 1] - (int64_t)s * P.r;
}

// The comparison method (paper Sec. II-B, Fig. 2): before step s of a round,
// chunk i takes the 2r planes of level s-1 just below its level-(s-1) area,
// [b_{i-1} - r(s+1), b_{i-1} - r(s-1)), from the sharing buffer (pool slot
// s-1, written by chunk i-1 during its own step s), then leaves its own
// top 2r planes of level s-1 there for chunk i+1, then runs one step.
static void build_resreu_chunk(const Plan &P, int t, int i, int kp, int slot,
                               std::vector<so2dr_op> &ops, int64_t *computed) {
  const int64_t r = P.r;
  so2dr_op base;
  std::memset(&base, 0, sizeof(base));
  base.round = t;
  base.chunk = i;
  base.slot = slot;
  base.buf_in = -1;
  base.buf_out = -1;
  base.buf_z0 = i == 0 ? 0 : P.bnd[i] - r * (P.K + 1);
  base.out_z0 = base.buf_z0;
  so2dr_op op = base;
  op.kind = SO2DR_OP_H2D;
  op.z0 = P.bnd[i];
  op.z1 = P.bnd[i + 1];
  op.buf_out = 0;
  ops.push_back(op);
  for (int st = 1; st <= kp; ++st) {
    const int in_buf = (st - 1) & 1;
    if (i > 0) {
      op = base;
      op.kind = SO2DR_OP_RS_READ;
      op.z0 = P.bnd[i] - r * (st + 1);
      op.z1 = P.bnd[i] - r * (st - 1);
      op.buf_out = in_buf;
      op.pool_off = 2 * r * (st - 1);
      ops.push_back(op);
    }
    if (i < P.d - 1) {
      op = base;
      op.kind = SO2DR_OP_RS_WRITE;
      op.z0 = P.bnd[i + 1] - r * (st + 1);
      op.z1 = P.bnd[i + 1] - r * (st - 1);
      op.buf_in = in_buf;
      op.pool_off = 2 * r * (st - 1);
      ops.push_back(op);
    }
    op = base;
    op.kind = SO2DR_OP_KERNEL;
    op.level_in = st - 1;
    op.levels = 1;
    op.in_z0 = i == 0 ? 0 : P.bnd[i] - r * (st + 1);
    op.in_z1 = area_hi(P, i, kp, st - 1);
    op.z0 = area_lo(P, i, kp, st);
    op.z1 = area_hi(P, i, kp, st);
    op.buf_in = in_buf;
    op.buf_out = st & 1;
    ops.push_back(op);
    *computed += op.z1 - op.z0;
  }
  op = base;
  op.kind = SO2DR_OP_D2H;
  op.z0 = area_lo(P, i, kp, kp);
  op.z1 = area_hi(P, i, kp, kp);
  op.buf_in = kp & 1;
  ops.push_back(op);
}

std::vector<so2dr_op> build_ops(const Plan &P, int steps, int64_t *planes_computed) {
  std::vector<so2dr_op> ops;
  int64_t computed = 0;
  const int nt = n_rounds_for(P, steps);
  for (int t = 0; t < nt; ++t) {
    const int kp = round_depth(P, steps, t);
    const int64_t h = 2 * (int64_t)P.r * kp;
    for (int i = 0; i < P.d; ++i) {
      const int slot = (int)(((int64_t)t * P.d + i) % P.n_slots);
      if (P.resreu) {
        build_resreu_chunk(P, t, i, kp, slot, ops, &computed);
        continue;
      }
      // the round-start data sits lean_extra planes above index 0 (lean plans)
      const int64_t buf_z0 = area_lo(P, i, kp, 0) - P.lean_extra;
      so2dr_op base;
      std::memset(&base, 0, sizeof(base));
      base.round = t;
      base.chunk = i;
      base.slot = slot;
      base.buf_in = -1;
      base.buf_out = -1;
      base.buf_z0 = buf_z0;
      base.out_z0 = buf_z0;
      // host -> slot buffer 0: the chunk's own planes
      so2dr_op op = base;
      op.kind = SO2DR_OP_H2D;
      op.z0 = P.bnd[i];
      op.z1 = P.bnd[i + 1];
      op.buf_out = 0;
      ops.push_back(op);
      // region sharing: read the lower halo, then write the own top
      if (i > 0) {
        op = base;
        op.kind = SO2DR_OP_RS_READ;
        op.z0 = P.bnd[i] - h;
        op.z1 = P.bnd[i];
        op.buf_out = 0;
        ops.push_back(op);
      }
      if (i < P.d - 1) {
        op = base;
        op.kind = SO2DR_OP_RS_WRITE;
        op.z0 = P.bnd[i + 1] - h;
        op.z1 = P.bnd[i + 1];
        op.buf_in = 0;
        ops.push_back(op);
      }
      // fused-step launches over the shrinking area
      int s = 0, j = 0;
      int64_t cur_z0 = buf_z0;  // global plane at index 0 of the data being read
      while (s < kp) {
        const int kl = std::min(P.k_on, kp - s);
        op = base;
        op.kind = SO2DR_OP_KERNEL;
        op.level_in = s;
        op.levels = kl;
        op.in_z0 = area_lo(P, i, kp, s);
        op.in_z1 = area_hi(P, i, kp, s);
        const int64_t o0 = area_lo(P, i, kp, s + kl), o1 = area_hi(P, i, kp, s + kl);
        if (!P.lean) {
          op.z0 = o0;
          op.z1 = o1;
          op.buf_in = j & 1;
          op.buf_out = (j + 1) & 1;
          op.buf_z0 = cur_z0;
          op.out_z0 = cur_z0;
          ops.push_back(op);
        } else {
          // one buffer: output sub-blocks of B planes in ascending order, each
          // written B + kl r planes below where it reads, i.e. over planes no
          // later sub-block reads (it needs planes >= its own start - kl r)
          const int64_t shift = P.lean_block + (int64_t)kl * P.r;
          op.buf_in = 0;
          op.buf_out = 0;
          op.buf_z0 = cur_z0;
          op.out_z0 = cur_z0 + shift;
          for (int64_t b = o0; b < o1; b += P.lean_block) {
            op.z0 = b;
            op.z1 = std::min(o1, b + (int64_t)P.lean_block);
            ops.push_back(op);
          }
          cur_z0 += shift;
        }
        for (int q = s + 1; q <= s + kl; ++q) computed += area_hi(P, i, kp, q) - area_lo(P, i, kp, q);
        s += kl;
        ++j;
      }
      // slot -> host: the output region
      op = base;
      op.kind = SO2DR_OP_D2H;
      op.z0 = area_lo(P, i, kp, kp);
      op.z1 = area_hi(P, i, kp, kp);
      op.buf_in = P.lean ? 0 : (j & 1);
      op.buf_z0 = cur_z0;
      ops.push_back(op);
    }
  }
  if (planes_computed) *planes_computed = computed;
  return ops;
}

// Byte total of a candidate (d, slots) plan; fills the sizes into P.  A lean
// plan keeps one buffer per slot with lean_extra spare planes below the data:
// every launch moves the data B + k r planes down while the valid area's
// bottom rises by k r (or not at all for the first chunk).
static size_t plan_bytes(Plan &P, int d, int slots, bool lean = false) {
  P.d = d;
  P.bnd.assign(d + 1, 0);
  for (int i = 0; i <= d; ++i) P.bnd[i] = (P.N * i) / d;
  const int64_t halo = d > 1 ? 2 * (int64_t)P.r * P.K : 0;
  // below its own planes a chunk holds the 2rK-plane shared halo, or for the
  // comparison method the r(K+1) planes its steps reach down to
  const int64_t below = d > 1 ? (P.resreu ? (int64_t)P.r * (P.K + 1) : halo) : 0;
  int64_t sp = 0;
  for (int i = 0; i < d; ++i) sp = std::max<int64_t>(sp, P.bnd[i + 1] - P.bnd[i] + (i > 0 ? below : 0));
  P.lean = lean;
  if (lean) {
    const int n_launch = (P.K + P.k_on - 1) / P.k_on;
    P.lean_block = (int)std::max<int64_t>(1, std::min<int64_t>(16, sp / 8));
    P.lean_extra = (int64_t)n_launch * P.lean_block + (int64_t)P.K * P.r;
    sp += P.lean_extra;
  } else {
    P.lean_block = 0;
    P.lean_extra = 0;
  }
  P.slot_planes = sp;
  P.buf_bytes = align256((size_t)sp * P.plane_bytes());
  P.rs_bytes = align256((size_t)halo * P.plane_bytes());
  P.n_slots = slots;
  // adjoint: per slot the round-start state and the adjoint field (copied in
  // while another slot computes), three working buffers (a recompute pair and
  // the adjoint's second buffer) shared by all slots since one stream
  // computes; a second region-sharing buffer for the adjoint field; FP64
  // partial sums for the loss and weight-gradient reductions
  P.bufs_per_slot = lean ? 1 : 2;
  P.shared_bufs = P.adjoint ? 3 : 0;
  P.scratch_bytes = P.adjoint ? align256(sizeof(double) * (kRedWgs * kMaxRedPts + 256)) : 0;
  return ((size_t)slots * P.bufs_per_slot + (size_t)P.shared_bufs) * P.buf_bytes +
         (size_t)P.n_rs() * P.rs_bytes + P.scratch_bytes;
}

static bool chunks_ok(const Plan &P, int d) {
  // every chunk but the last hands its top 2 r K planes to the next one, so
  // it must own at least that many (paper: halo space <= chunk)
  if (d < 1 || d > P.N) return false;
  if (d == 1) return true;
  // the comparison method shares r(s+1)..r(s-1) below level s: it needs the
  // chunk to own r(K+1) planes so its level-K area stays inside it
  const int64_t halo = P.resreu ? (int64_t)P.r * (P.K + 1) : 2 * (int64_t)P.r * P.K;
  for (int i = 0; i + 1 < d; ++i)
    if ((P.N * (i + 1)) / d - (P.N * i) / d < halo) return false;
  return true;
}

int make_plan(const so2dr_desc &D, Plan *P) {
  if (D.ndim != 2 && D.ndim != 3) { set_error("ndim must be 2 or 3"); return SO2DR_E_INVALID; }
  if (D.nx < 1 || D.ny < 1 || D.nz < 1) { set_error("grid extents must be >= 1"); return SO2DR_E_INVALID; }
  if (D.ndim == 2 && D.nz != 1) { set_error("a 2D grid has nz == 1"); return SO2DR_E_INVALID; }
  if (D.shape != SO2DR_STAR && D.shape != SO2DR_BOX) { set_error("unknown stencil shape"); return SO2DR_E_INVALID; }
  if (D.radius < 1) { set_error("radius must be >= 1"); return SO2DR_E_INVALID; }
  if (dtype_size(D.storage) == 0) { set_error("unknown storage type"); return SO2DR_E_INVALID; }
  if (!D.weights || D.n_weights != expected_points(D.ndim, D.shape, D.radius)) {
    set_error("n_weights does not match the stencil's point count");
    return SO2DR_E_INVALID;
  }
  for (int a = 0; a < 3; ++a)
    if (D.bc[a] != SO2DR_DIRICHLET0 && D.bc[a] != SO2DR_PERIODIC) { set_error("unknown boundary rule"); return SO2DR_E_INVALID; }
  if (D.T < 0 || D.tb_depth < 0 || D.k_on < 0 || D.n_chunks < 0 || D.n_slots < 0 || D.n_slots > 4) {
    set_error("negative T/tb_depth/k_on/n_chunks or n_slots > 4");
    return SO2DR_E_INVALID;
  }
  P->ndim = D.ndim;
  P->shape = D.shape;
  P->r = D.radius;
  P->dtype = D.storage;
  P->nx = D.nx;
  P->ny = D.ny;
  P->nz = D.nz;
  P->elem = dtype_size(D.storage);
  if (D.ndim == 3) {
    P->NX = D.nx; P->NY = D.ny; P->N = D.nz;
    P->per_x = D.bc[0] == SO2DR_PERIODIC;
    P->per_y = D.bc[1] == SO2DR_PERIODIC;
    if (D.bc[2] != SO2DR_DIRICHLET0) { set_error("the cut axis (z) must be zero Dirichlet"); return SO2DR_E_UNSUPPORTED; }
  } else {
    P->NX = D.nx; P->NY = 1; P->N = D.ny;
    P->per_x = D.bc[0] == SO2DR_PERIODIC;
    P->per_y = 0;
    if (D.bc[1] != SO2DR_DIRICHLET0) { set_error("the cut axis (y) must be zero Dirichlet"); return SO2DR_E_UNSUPPORTED; }
  }
  if (P->NX > (1 << 30) || P->NY > (1 << 30) || P->NX * P->NY > ((int64_t)1 << 31)) {
    set_error("plane too large");
    return SO2DR_E_UNSUPPORTED;
  }
  P->plane = P->NX * P->NY;
  P->weights.assign(D.weights, D.weights + D.n_weights);
  for (double w : P->weights)
    if (!std::isfinite(w)) { set_error("weights must be finite"); return SO2DR_E_INVALID; }
  P->stencil = stencil_id(D.ndim, D.shape, D.radius);
  P->max_k_on = max_depth(D.storage, P->stencil);
  if (P->stencil < 0 || P->max_k_on == 0) {
    set_error("no kernel built for this stencil and storage type");
    return SO2DR_E_UNSUPPORTED;
  }
  P->T = D.T;
  P->K = D.tb_depth == 0 ? std::max(1, D.T) : std::min(D.tb_depth, std::max(1, D.T));
  if (D.k_on > 0) {
    if (D.k_on > P->max_k_on) {
      set_error("k_on deeper than the deepest fused kernel built for this stencil");
      return SO2DR_E_UNSUPPORTED;
    }
    P->k_on = std::min(D.k_on, P->K);
  } else {
    // the fused depth with the best measured update rate per launch on
    // MI355X for this stencil and storage type (rates.hpp): e.g. FP32 3 for
    // the 7-point star, 2 for the 13-point star and the 27-point box, 8 for
    // the 2D 5-point star, 1 for the widest boxes (bound by arithmetic:
    // fusing only adds tile-edge recomputation)
    const int pref = preferred_depth(P->dtype, P->stencil, P->max_k_on);
    P->k_on = std::max(1, std::min(pref, P->K));
  }
  P->budget = D.device_budget_bytes;
  P->adjoint = D.adjoint != 0;
  if (D.method != SO2DR_METHOD_SO2DR && D.method != SO2DR_METHOD_RESREU) {
    set_error("unknown method");
    return SO2DR_E_INVALID;
  }
  P->resreu = D.method == SO2DR_METHOD_RESREU;
  if (D.rounding != SO2DR_ROUND_EVERY_STEP && D.rounding != SO2DR_ROUND_AT_STORE) {
    set_error("unknown rounding mode");
    return SO2DR_E_INVALID;
  }
  P->ras = D.rounding == SO2DR_ROUND_AT_STORE && (P->dtype == SO2DR_BF16 || P->dtype == SO2DR_F16);
  if (D.copy_engine < SO2DR_COPY_AUTO || D.copy_engine > SO2DR_COPY_KERNEL_OUT) {
    set_error("unknown copy engine");
    return SO2DR_E_INVALID;
  }
  if (P->resreu) {
    if (P->adjoint) {
      set_error("the comparison method has no adjoint");
      return SO2DR_E_UNSUPPORTED;
    }
    P->k_on = 1;  // its kernels can only advance one step (Sec. III)
  }
  // ---- chunk count and slots
  if (D.n_chunks > 0) {
    if (!chunks_ok(*P, D.n_chunks)) {
      set_error("n_chunks too large: a chunk must own at least 2*radius*tb_depth planes");
      return SO2DR_E_INVALID;
    }
    int want = D.n_slots > 0 ? D.n_slots : std::min(3, D.n_chunks);
    int slots = want;
    while (slots >= 1 && plan_bytes(*P, D.n_chunks, slots) > P->budget) {
      if (D.n_slots > 0) { slots = 0; break; }
      --slots;
    }
    bool lean = false;
    if (slots < 1 && !P->adjoint && !P->resreu) {  // one buffer per slot instead of two
      slots = want;
      while (slots >= 1 && plan_bytes(*P, D.n_chunks, slots, true) > P->budget) {
        if (D.n_slots > 0) { slots = 0; break; }
        --slots;
      }
      lean = slots >= 1;
    }
    if (slots < 1) {
      set_error("plan does not fit the device budget (chunks " + std::to_string(D.n_chunks) + ")");
      return SO2DR_E_BUDGET;
    }
    plan_bytes(*P, D.n_chunks, slots, lean);
  } else {
    // fewest chunks that fit with min(3, d) slots; else the fewest that fit at all
    int chosen = 0, chosen_slots = 0;
    for (int pass = 0; pass < 2 && !chosen; ++pass) {
      for (int d = 1; d <= P->N && !chosen; ++d) {
        if (!chunks_ok(*P, d)) break;
        const int want = D.n_slots > 0 ? D.n_slots : std::min(3, d);
        for (int slots = want; slots >= (pass == 0 ? want : 1); --slots)
          if (plan_bytes(*P, d, slots) <= P->budget) { chosen = d; chosen_slots = slots; break; }
      }
    }
    bool lean = false;
    for (int d = 1; !chosen && !P->adjoint && !P->resreu && d <= P->N; ++d) {  // lean as a last resort
      if (!chunks_ok(*P, d)) break;
      for (int slots = D.n_slots > 0 ? D.n_slots : std::min(3, d); slots >= 1; --slots)
        if (plan_bytes(*P, d, slots, true) <= P->budget) { chosen = d; chosen_slots = slots; lean = true; break; }
    }
    if (!chosen) { set_error("no chunk count fits the device budget"); return SO2DR_E_BUDGET; }
    plan_bytes(*P, chosen, chosen_slots, lean);
  }
  P->workspace = ((size_t)P->n_slots * P->bufs_per_slot + (size_t)P->shared_bufs) * P->buf_bytes +
                 (size_t)P->n_rs() * P->rs_bytes + P->scratch_bytes;
  // Copy engine.  Measured on MI355X with everything enqueued at once, DMA
  // copies ran at the link's 97 GB/s only while each copy was large; with
  // smaller copies the rate became erratic (a 64 MiB pattern: 28-82 GB/s
  // over repeats) while copy kernels held 84-86 GB/s at any size; DMA in with
  // copy kernels out did best in the executor (the 7-point workload at 32
  // chunks: 88 GB/s, against 77 with kernels both ways).  Few queued
  // copies stay fast on DMA (the 27-point workload at 32 chunks and two
  // rounds: 190 GCell/s), so the count queued by one run counts too.  Adjoint
  // plans keep DMA: their reverse sweep waits for each round and its compute
  // kernels compete with copy kernels (the 1024^3 gradient: 4.9 s with DMA,
  // 7.2 s with copy kernels).
  P->copy_engine_forced = D.copy_engine != SO2DR_COPY_AUTO;
  if (P->copy_engine_forced) {
    P->copy_engine = D.copy_engine;
  } else {
    int64_t own = 0;
    for (int i = 0; i < P->d; ++i) own = std::max<int64_t>(own, P->bnd[i + 1] - P->bnd[i]);
    const int64_t rounds = P->K > 0 ? (P->T + P->K - 1) / P->K : 1;
    const int64_t queued = 2 * (int64_t)P->d * rounds;
    P->copy_engine = !P->adjoint && (size_t)own * P->plane_bytes() < kKernelCopyBelow && queued > kKernelCopyQueued
                         ? SO2DR_COPY_KERNEL_OUT
                         : SO2DR_COPY_DMA;
  }
  return SO2DR_OK;
}

}  // namespace so2dr
