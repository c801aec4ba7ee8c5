// adjoint.cpp -- reverse-mode gradient of the out-of-core sweep.
//
// Not in the paper: the paper's sweep is forward only.  For
//   L = 1/2 sum_x (u_T(x) - y(x))^2,   u_{t+1} = A u_t  (A = the stencil),
// the chain rule gives lambda_T = u_T - y, lambda_t = A^T lambda_{t+1},
// dL/du_0 = lambda_0 and dL/dw_k = sum_t sum_x lambda_{t+1}(x) u_t(x + o_k).
// A^T is the correlation with the reflected point set: for the symmetric
// star and box sets, negating an offset reverses its lexicographic rank, so
// A^T runs the forward kernels with the weight array reversed.
//
// Schedule (all out of core, same chunking and region sharing as forward):
//   1. forward in segments of ckpt_every steps, each segment's start state
//      kept in a caller-owned pinned host buffer; u_T lands in grad_u0;
//   2. loss pass: per chunk, lambda_T = u_T - y in place and 1/2 (u - y)^2
//      summed in FP64 on the GPU;
//   3. per segment, last first: recompute the states at the segment's round
//      starts (forward rounds of tb_depth steps) from its checkpoint, then
//      run reverse rounds, last first.  A reverse round over steps
//      [t_s, t_e) streams each chunk's u_{t_s} and lambda_{t_e} (own planes
//      from the host, the 2 r k' planes below from the two region-sharing
//      buffers), recomputes u_t on the shrinking areas of the forward round,
//      steps lambda back with A^T on the same areas, and adds
//      lambda_{t+1}(x) u_t(x + o_k) over the planes the chunk owns,
//      [b_{i-1} - r k', b_i - r k'), which partition the grid and lie inside
//      every level's valid area.  lambda_{t_s} goes back to the host in place.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "aux.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace so2dr {

int execute(Plan &P, const void *host_in, void *host_out, int steps, so2dr_stats *st);
int check_pinned(const void *p, size_t bytes, const char *what);

#define AHIP(expr)                                                                    \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));                   \
      return SO2DR_E_HIP;                                                             \
    }                                                                                 \
  } while (0)

#define ARC(expr)            \
  do {                       \
    const int rc_ = (expr);  \
    if (rc_) return rc_;     \
  } while (0)

static int ensure(std::vector<hipEvent_t> &v, size_t n) {
  while (v.size() < n) {
    hipEvent_t e;
    AHIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    v.push_back(e);
  }
  return SO2DR_OK;
}

// Offsets of the plan's stencil in lexicographic order, in the internal
// (cut axis, in-plane y, x) frame: a 2D stencil's (dy, dx) acts as (dz, 0, dx).
static RedOffsets internal_offsets(const Plan &P, int *npts) {
  RedOffsets o;
  std::memset(&o, 0, sizeof(o));
  const int r = P.r;
  int k = 0;
  for (int a = (P.ndim == 3 ? -r : 0); a <= (P.ndim == 3 ? r : 0); ++a)
    for (int b = -r; b <= r; ++b)
      for (int c = -r; c <= r; ++c) {
        const int nz = (a != 0) + (b != 0) + (c != 0);
        if (P.shape == SO2DR_STAR && nz > 1) continue;
        if (P.ndim == 3) {
          o.dz[k] = (int8_t)a;
          o.dy[k] = (int8_t)b;
        } else {
          o.dz[k] = (int8_t)b;
          o.dy[k] = 0;
        }
        o.dx[k] = (int8_t)c;
        ++k;
      }
  *npts = k;
  return o;
}

static LaunchParams base_launch(const Plan &P, const double *w) {
  LaunchParams lp;
  std::memset(&lp, 0, sizeof(lp));
  lp.stencil = P.stencil;
  lp.plane = P.plane;
  lp.nx = (int)P.NX;
  lp.ny = (int)P.NY;
  lp.per_x = P.per_x;
  lp.per_y = P.per_y;
  lp.n_axis = P.N;
  lp.weights = w;
  lp.npts = (int)P.weights.size();
  return lp;
}

struct AdjCtx {
  hipStream_t s_in, s_out, s_comp;
  bool kcopy = false;  // HBM -> host copies by copy kernels through the host mappings
  bool kcopy_in = false;  // host -> HBM copies too
  size_t field = 0;
  double *partials, *acc_w, *acc_loss;
  std::vector<double> wT;  // reflected weights
  RedOffsets offs;
  int npts;
};

// Loss pass over the chunks (no halo): lam_host holds u_T and becomes lambda_T.
static int loss_pass(Plan &P, AdjCtx &C, void *lam_host, const void *y_host, so2dr_stats *S) {
  const size_t pb = P.plane_bytes();
  ARC(ensure(P.ev_h2d, P.d));
  ARC(ensure(P.ev_comp, P.d));
  ARC(ensure(P.ev_d2h, P.d));
  char *d_lam = C.kcopy ? mapped_host(lam_host, C.field) : nullptr;
  char *d_lam_in = C.kcopy_in ? d_lam : nullptr;
  char *d_y = C.kcopy_in ? mapped_host(y_host, C.field) : nullptr;
  for (int i = 0; i < P.d; ++i) {
    const int slot = i % P.n_slots;
    const int64_t z0 = P.bnd[i], z1 = P.bnd[i + 1];
    const size_t n = (size_t)(z1 - z0) * pb;
    char *ub = P.slot_buf(slot, 0), *yb = P.slot_buf(slot, 1);
    if (i >= P.n_slots) AHIP(hipStreamWaitEvent(C.s_in, P.ev_d2h[i - P.n_slots], 0));
    ARC(copy_to_device(ub, static_cast<char *>(lam_host) + (size_t)z0 * pb, n, lam_host, d_lam_in, C.s_in));
    ARC(copy_to_device(yb, static_cast<const char *>(y_host) + (size_t)z0 * pb, n, y_host, d_y, C.s_in));
    AHIP(hipEventRecord(P.ev_h2d[i], C.s_in));
    AHIP(hipStreamWaitEvent(C.s_comp, P.ev_h2d[i], 0));
    if (launch_loss(P.dtype, ub, yb, (int64_t)(z1 - z0) * P.plane, C.partials, C.acc_loss, C.s_comp)) {
      set_error("loss kernel launch failed");
      return SO2DR_E_HIP;
    }
    AHIP(hipEventRecord(P.ev_comp[i], C.s_comp));
    AHIP(hipStreamWaitEvent(C.s_out, P.ev_comp[i], 0));
    ARC(copy_to_host(static_cast<char *>(lam_host) + (size_t)z0 * pb, ub, n, lam_host, d_lam, C.s_out));
    AHIP(hipEventRecord(P.ev_d2h[i], C.s_out));
    S->bytes_h2d += 2 * n;
    S->bytes_d2h += n;
  }
  AHIP(hipStreamSynchronize(C.s_in));
  AHIP(hipStreamSynchronize(C.s_comp));
  AHIP(hipStreamSynchronize(C.s_out));
  return SO2DR_OK;
}

// One reverse round of depth kp: lam_host goes from lambda_{t_e} to
// lambda_{t_s} in place; u_host holds u_{t_s}.
static int reverse_round(Plan &P, AdjCtx &C, const void *u_host, void *lam_host, int kp,
                         so2dr_stats *S) {
  // per slot: round-start u and lambda; shared: u recompute pair, lambda's
  // second buffer
  enum { U0 = 0, LA = 1, UA = 2, UB = 3, LB = 4 };
  const size_t pb = P.plane_bytes();
  const int64_t h = 2 * (int64_t)P.r * kp;
  ARC(ensure(P.ev_h2d, P.d));
  ARC(ensure(P.ev_comp, P.d));
  ARC(ensure(P.ev_d2h, P.d));
  ARC(ensure(P.ev_rs, P.d));
  std::string msg;
  char *d_u = C.kcopy_in ? mapped_host(u_host, C.field) : nullptr;
  char *d_lam = C.kcopy ? mapped_host(lam_host, C.field) : nullptr;
  char *d_lam_in = C.kcopy_in ? d_lam : nullptr;
  LaunchParams fwd = base_launch(P, P.weights.data());
  LaunchParams adj = base_launch(P, C.wT.data());
  for (int i = 0; i < P.d; ++i) {
    const int slot = i % P.n_slots;
    const int64_t b0 = P.bnd[i], b1 = P.bnd[i + 1];
    const int64_t bz = area_lo(P, i, kp, 0);
    auto buf = [&](int which) { return P.slot_buf(slot, which); };
    auto at = [&](int which, int64_t z) { return buf(which) + (size_t)(z - bz) * pb; };
    // copy-in of the own planes of u_{t_s} and lambda_{t_e}
    if (i >= P.n_slots) AHIP(hipStreamWaitEvent(C.s_in, P.ev_d2h[i - P.n_slots], 0));
    const size_t own = (size_t)(b1 - b0) * pb;
    ARC(copy_to_device(at(U0, b0), static_cast<const char *>(u_host) + (size_t)b0 * pb, own, u_host, d_u,
                       C.s_in));
    ARC(copy_to_device(at(LA, b0), static_cast<char *>(lam_host) + (size_t)b0 * pb, own, lam_host, d_lam_in,
                       C.s_in));
    AHIP(hipEventRecord(P.ev_h2d[i], C.s_in));
    S->bytes_h2d += 2 * own;
    // region sharing for both fields: read the lower halo, then write the own top
    hipStream_t s = C.s_comp;
    AHIP(hipStreamWaitEvent(s, P.ev_h2d[i], 0));
    if (i > 0) AHIP(hipStreamWaitEvent(s, P.ev_rs[i - 1], 0));
    for (int f = 0; f < 2; ++f) {
      const int which = f == 0 ? U0 : LA;
      // copy kernels on the compute stream, as in the forward executor
      if ((i > 0 && launch_dcopy(at(which, b0 - h), P.rs_pool(f), (size_t)h * pb, s)) ||
          (i < P.d - 1 && launch_dcopy(P.rs_pool(f), at(which, b1 - h), (size_t)h * pb, s))) {
        set_error("region-sharing copy kernel launch failed");
        return SO2DR_E_HIP;
      }
      S->bytes_d2d += (size_t)h * pb * ((i > 0) + (i < P.d - 1));
    }
    AHIP(hipEventRecord(P.ev_rs[i], s));
    const int64_t own_lo = i == 0 ? 0 : b0 - (int64_t)P.r * kp;
    const int64_t own_hi = i == P.d - 1 ? P.N : b1 - (int64_t)P.r * kp;
    int lcur = LA, lnext = LB;
    for (int st = 0; st < kp; ++st) {
      const int m = kp - 1 - st;  // u level paired with lambda level st
      int ubuf = U0;
      if (m > 0) {  // recompute u level m from the round-start state
        int src = U0, dst = UA, done = 0;
        while (done < m) {
          const int kl = std::min(P.k_on, m - done);
          LaunchParams lp = fwd;
          lp.kl = kl;
          lp.in = buf(src);
          lp.out = buf(dst);
          lp.buf_z0 = bz;
          lp.out_z0 = bz;
          lp.in_lo = area_lo(P, i, kp, done);
          lp.in_hi = area_hi(P, i, kp, done);
          lp.out_lo = area_lo(P, i, kp, done + kl);
          lp.out_hi = area_hi(P, i, kp, done + kl);
          const int rc = launch_tb(P.dtype, lp, s, &msg);
          if (rc) {
            set_error(msg);
            return rc;
          }
          S->kernel_launches += 1;
          done += kl;
          src = dst;
          dst = dst == UA ? UB : UA;
        }
        ubuf = src;
      }
      // dL/dw_k += sum over owned planes of lambda_{t+1}(x) u_t(x + o_k)
      if (launch_wgrad(P.dtype, buf(lcur), buf(ubuf), bz, (int)P.NX, (int)P.NY, P.per_x, P.per_y, P.N,
                       own_lo, own_hi, C.offs, C.npts, C.partials, C.acc_w, s)) {
        set_error("weight-gradient kernel launch failed");
        return SO2DR_E_HIP;
      }
      // lambda_t = A^T lambda_{t+1} on the next, smaller area
      LaunchParams lp = adj;
      lp.kl = 1;
      lp.in = buf(lcur);
      lp.out = buf(lnext);
      lp.buf_z0 = bz;
      lp.out_z0 = bz;
      lp.in_lo = area_lo(P, i, kp, st);
      lp.in_hi = area_hi(P, i, kp, st);
      lp.out_lo = area_lo(P, i, kp, st + 1);
      lp.out_hi = area_hi(P, i, kp, st + 1);
      const int rc = launch_tb(P.dtype, lp, s, &msg);
      if (rc) {
        set_error(msg);
        return rc;
      }
      S->kernel_launches += 1;
      std::swap(lcur, lnext);
    }
    // copy-out of lambda_{t_s} over the chunk's output planes, in place, from
    // the slot's own buffer: the shared one is the next chunk's
    const int64_t o0 = area_lo(P, i, kp, kp), o1 = area_hi(P, i, kp, kp);
    if (lcur != LA) {
      if (launch_dcopy(at(LA, o0), at(lcur, o0), (size_t)(o1 - o0) * pb, s)) {
        set_error("adjoint copy kernel launch failed");
        return SO2DR_E_HIP;
      }
      lcur = LA;
    }
    AHIP(hipEventRecord(P.ev_comp[i], s));
    AHIP(hipStreamWaitEvent(C.s_out, P.ev_comp[i], 0));
    ARC(copy_to_host(static_cast<char *>(lam_host) + (size_t)o0 * pb, at(lcur, o0), (size_t)(o1 - o0) * pb,
                     lam_host, d_lam, C.s_out));
    AHIP(hipEventRecord(P.ev_d2h[i], C.s_out));
    S->bytes_d2h += (size_t)(o1 - o0) * pb;
  }
  AHIP(hipStreamSynchronize(C.s_in));
  AHIP(hipStreamSynchronize(C.s_comp));
  AHIP(hipStreamSynchronize(C.s_out));
  return SO2DR_OK;
}

static int adjoint_impl(Plan &P, const void *u0, const void *target, void *grad_u0, double *grad_w,
                        double *loss, int ckpt_every, void *const *ckpt, int n_ckpt, so2dr_stats *st) {
  if (!P.bound) {
    set_error("plan is not bound to device memory and streams");
    return SO2DR_E_UNBOUND;
  }
  if (!P.adjoint) {
    set_error("plan was created without adjoint = 1 (no device space reserved)");
    return SO2DR_E_INVALID;
  }
  if (P.dtype != SO2DR_F32 && P.dtype != SO2DR_F64) {
    set_error("the adjoint is built for F32 and F64 storage");
    return SO2DR_E_UNSUPPORTED;
  }
  if (!grad_w || !loss || ckpt_every < 1) {
    set_error("null grad_w/loss or ckpt_every < 1");
    return SO2DR_E_INVALID;
  }
  const int T = P.T;
  const int c = std::min(ckpt_every, std::max(T, 1));
  const int nseg = T > 0 ? (T + c - 1) / c : 0;
  const int n_scratch = std::max(0, (c + P.K - 1) / P.K - 1);
  const int need = std::max(0, nseg - 1) + n_scratch;
  if (n_ckpt < need || (need > 0 && !ckpt)) {
    set_error("need " + std::to_string(need) + " host checkpoint buffers (segments - 1 + ceil(ckpt_every / tb_depth) - 1)");
    return SO2DR_E_INVALID;
  }
  const size_t field = (size_t)P.N * P.plane_bytes();
  ARC(check_pinned(u0, field, "u0"));
  ARC(check_pinned(target, field, "target"));
  ARC(check_pinned(grad_u0, field, "grad_u0"));
  for (int j = 0; j < need; ++j) ARC(check_pinned(ckpt[j], field, "checkpoint buffer"));

  so2dr_stats S;
  std::memset(&S, 0, sizeof(S));
  const auto t0 = std::chrono::steady_clock::now();
  AdjCtx C;
  C.field = field;
  C.kcopy = P.copy_engine == SO2DR_COPY_KERNEL || P.copy_engine == SO2DR_COPY_KERNEL_OUT;
  C.kcopy_in = P.copy_engine == SO2DR_COPY_KERNEL;
  if (C.kcopy) {
    bool all = mapped_host(u0, field) && mapped_host(target, field) && mapped_host(grad_u0, field);
    for (int j = 0; j < need; ++j) all = all && mapped_host(ckpt[j], field);
    if (!all) {
      if (P.copy_engine_forced) {
        set_error("copy kernels need each host array inside one page-locked allocation mapped into the device");
        return SO2DR_E_NOT_PINNED;
      }
      C.kcopy = C.kcopy_in = false;
    }
  }
  const int ns = (int)P.streams.size();
  C.s_in = P.streams[0];
  C.s_out = ns >= 2 ? P.streams[1] : P.streams[0];
  C.s_comp = ns >= 3 ? P.streams[2] : P.streams[0];
  C.partials = reinterpret_cast<double *>(P.scratch());
  C.acc_w = C.partials + (size_t)kRedWgs * kMaxRedPts;
  C.acc_loss = C.acc_w + 128;
  C.wT.assign(P.weights.rbegin(), P.weights.rend());
  C.offs = internal_offsets(P, &C.npts);
  if (C.npts != (int)P.weights.size()) {
    set_error("internal offset enumeration does not match the weight count");
    return SO2DR_E_INVALID;
  }
  AHIP(hipMemsetAsync(C.acc_w, 0, sizeof(double) * 129, C.s_comp));

  auto state = [&](int j) -> const void * { return j == 0 ? u0 : ckpt[j - 1]; };
  // 1. forward, keeping segment starts; u_T lands in grad_u0
  for (int j = 0; j < nseg; ++j) {
    const int len = std::min(c, T - j * c);
    void *dst = j == nseg - 1 ? grad_u0 : ckpt[j];
    so2dr_stats fs;
    ARC(execute(P, state(j), dst, len, &fs));
    S.bytes_h2d += fs.bytes_h2d;
    S.bytes_d2h += fs.bytes_d2h;
    S.bytes_d2d += fs.bytes_d2d;
    S.kernel_launches += fs.kernel_launches;
  }
  if (T == 0) std::memcpy(grad_u0, u0, field);
  // 2. loss and lambda_T
  ARC(loss_pass(P, C, grad_u0, target, &S));
  // 3. reverse, segment by segment
  for (int j = nseg - 1; j >= 0; --j) {
    const int len = std::min(c, T - j * c);
    const int nr = (len + P.K - 1) / P.K;
    std::vector<const void *> starts(nr);
    starts[0] = state(j);
    for (int m = 1; m < nr; ++m) {
      void *dst = ckpt[std::max(0, nseg - 1) + m - 1];
      so2dr_stats fs;
      ARC(execute(P, starts[m - 1], dst, P.K, &fs));
      S.bytes_h2d += fs.bytes_h2d;
      S.bytes_d2h += fs.bytes_d2h;
      S.kernel_launches += fs.kernel_launches;
      starts[m] = dst;
    }
    for (int m = nr - 1; m >= 0; --m) {
      const int kp = m == nr - 1 ? len - (nr - 1) * P.K : P.K;
      ARC(reverse_round(P, C, starts[m], grad_u0, kp, &S));
    }
  }
  double host_acc[129];
  AHIP(hipMemcpyAsync(host_acc, C.acc_w, sizeof(host_acc), hipMemcpyDeviceToHost, C.s_comp));
  AHIP(hipStreamSynchronize(C.s_comp));
  for (int k = 0; k < C.npts; ++k) grad_w[k] = host_acc[k];
  *loss = host_acc[128];
  S.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  S.cell_updates = (uint64_t)P.N * (uint64_t)P.plane * (uint64_t)T;
  S.rounds_done = nseg;
  if (st) *st = S;
  return SO2DR_OK;
}

// On a failure part-way the work already queued is drained before
// returning, so the caller may release the arena and host buffers at once.
int adjoint_run(Plan &P, const void *u0, const void *target, void *grad_u0, double *grad_w,
                double *loss, int ckpt_every, void *const *ckpt, int n_ckpt, so2dr_stats *st) {
  const int rc = adjoint_impl(P, u0, target, grad_u0, grad_w, loss, ckpt_every, ckpt, n_ckpt, st);
  if (rc && P.bound) drain_streams(P);
  return rc;
}

}  // namespace so2dr
