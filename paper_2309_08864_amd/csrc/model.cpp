// model.cpp -- a cost model of a plan's run and a planner that searches the
// free plan parameters with it (the automatic choice of chunk count, TB depth
// and fused steps that the paper leaves to future work, Sec. IV-C / VII).
//
// The model replays the plan's own schedule (build_ops) through the
// executor's dependency rules (schedule_deps, the code the executor runs:
// copy-in and copy-out streams in order, one compute stream, slot reuse,
// region-sharing order, host hazards between rounds) with each operation's
// duration taken from machine figures: host
// link rates (solo and full duplex), device copy rate, fixed launch cost and
// the measured update rate of a fused launch per depth.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "plan.hpp"
#include "rates.hpp"

namespace so2dr {

int max_depth(int dtype, int stencil);

namespace {

struct Sim {
  double bw_in, bw_out, bw_d2d, launch_s;
};

}  // namespace

void default_machine(const Plan &P, so2dr_machine *m) {
  std::memset(m, 0, sizeof(*m));
  // pinned hipMemcpyAsync on the MI355X machine: each direction alone, both at once
  m->h2d_gbps = 57.3;
  m->d2h_gbps = 57.0;
  m->duplex_gbps = 97.3;
  m->d2d_gbps = 2000.0;
  m->launch_us = 8.0;
  m->kcopy_gbps = 77.0;      // copy kernels of 64 workgroups both ways, beside stencil kernels
  m->kcopy_out_gbps = 88.0;  // DMA in, copy kernels out
  // measured per storage type, stencil and depth (rates.hpp)
  const int md = max_depth(P.dtype, P.stencil);
  for (int k = 1; k <= 8; ++k) m->gupd[k - 1] = k <= md ? kernel_rate(P.dtype, P.stencil, k) : 0.0;
}

namespace {

double simulate(const Plan &P, const so2dr_machine &m, int steps) {
  int64_t computed = 0;
  const std::vector<so2dr_op> ops = build_ops(P, steps, &computed);
  // the executor's own stream assignment and waits, for the library's
  // three streams (copy-in, copy-out, compute)
  std::vector<int> strm;
  std::vector<int64_t> waits;
  schedule_deps(P, ops, 3, &strm, &waits);
  // with two or more slots both copy directions run together most of the time
  const bool duplex = P.n_slots >= 2;
  double both = m.duplex_gbps;
  if (P.copy_engine == SO2DR_COPY_KERNEL && m.kcopy_gbps > 0) both = m.kcopy_gbps;
  if (P.copy_engine == SO2DR_COPY_KERNEL_OUT && m.kcopy_out_gbps > 0) both = m.kcopy_out_gbps;
  Sim S;
  S.bw_in = 1e9 * (duplex ? std::min(m.h2d_gbps, 0.5 * both) : m.h2d_gbps);
  S.bw_out = 1e9 * (duplex ? std::min(m.d2h_gbps, 0.5 * both) : m.d2h_gbps);
  S.bw_d2d = 1e9 * m.d2d_gbps;
  S.launch_s = 1e-6 * m.launch_us;
  const size_t pb = P.plane_bytes();
  std::vector<double> end(ops.size(), 0.0);
  double stream_end[3] = {0.0, 0.0, 0.0}, t_end = 0.0;
  for (size_t k = 0; k < ops.size(); ++k) {
    const so2dr_op &op = ops[k];
    const double bytes = (double)(op.z1 - op.z0) * (double)pb;
    double start = stream_end[strm[k]];
    for (int i = 0; i < kMaxWaits; ++i) {
      const int64_t w = waits[k * kMaxWaits + i];
      if (w >= 0) start = std::max(start, end[(size_t)w]);
    }
    double dur = 0.0;
    switch (op.kind) {
      case SO2DR_OP_H2D: dur = bytes / S.bw_in; break;
      case SO2DR_OP_D2H: dur = bytes / S.bw_out; break;
      case SO2DR_OP_KERNEL: {
        const double rate = op.levels >= 1 && op.levels <= 8 ? m.gupd[op.levels - 1] : 0.0;
        const double upd = (double)(op.z1 - op.z0) * (double)P.plane * op.levels;
        dur = S.launch_s + (rate > 0 ? upd / (rate * 1e9) : 1e30);
        break;
      }
      default: dur = 2.0 * bytes / S.bw_d2d + S.launch_s; break;   // region-sharing copies
    }
    end[k] = start + dur;
    stream_end[strm[k]] = end[k];
    t_end = std::max(t_end, end[k]);
  }
  return t_end;
}

}  // namespace

// Rounds after the second repeat the same pattern, so a long run is
// simulated for three rounds and extrapolated by the per-round increment.
double predict_seconds(const Plan &P, const so2dr_machine &m, int steps) {
  const int K = std::max(P.K, 1);
  const int full = steps / K, rem = steps % K;
  if (full <= 3) return simulate(P, m, steps);
  const double t2 = simulate(P, m, 2 * K), t3 = simulate(P, m, 3 * K);
  double t = t3 + (double)(full - 3) * (t3 - t2);
  if (rem > 0) t += simulate(P, m, 3 * K + rem) - t3;
  return t;
}

namespace {

// Chunk counts searched.  Measured on MI355X, many small host copies run
// slower than the model's link figures: DMA copies collapse when hundreds are
// queued (the reason for the copy-kernel modes), and even DMA in with copy
// kernels out fell from 88 to 69 GB/s at 64 chunks of the 7-point workload.
// So the search stops at 32 chunks and takes a candidate with more chunks,
// more fused levels or a deeper round only when it is predicted more than
// 1 % faster (candidates are visited in increasing order).
constexpr int64_t kMaxSearchChunks = 32;
constexpr double kMinGain = 0.01;

std::vector<int> depth_candidates(int T) {
  static const int base[] = {1,   2,   3,   4,   5,   6,   8,   10,  12,  16,   20,   24,  32,
                             40,  48,  64,  80,  96,  128, 160, 192, 256, 320, 384, 512, 640,
                             768, 1024, 1280, 1536, 2048, 2560, 3072, 4096};
  std::vector<int> out;
  for (int k : base)
    if (k <= T) out.push_back(k);
  if (T >= 1 && (out.empty() || out.back() != T)) out.push_back(T);
  return out;
}

}  // namespace

int suggest(const so2dr_desc &in, const so2dr_machine *mp, so2dr_desc *out, double *pred_ms) {
  // validate the problem itself (stencil, storage, extents) without the
  // budget; this also gives the stencil id for the machine figures
  Plan base;
  so2dr_desc c0 = in;
  c0.tb_depth = 1;
  c0.k_on = 1;
  c0.n_chunks = 0;
  c0.n_slots = 0;
  c0.device_budget_bytes = (size_t)1 << 62;
  int rc = make_plan(c0, &base);
  if (rc) return rc;
  so2dr_machine m;
  if (mp) m = *mp; else default_machine(base, &m);
  const int T = in.T;
  const std::vector<int> Ks = in.tb_depth > 0 ? std::vector<int>{std::min(in.tb_depth, std::max(T, 1))}
                                              : depth_candidates(std::max(T, 1));
  double best = -1;
  so2dr_desc best_d = in;
  for (int K : Ks) {
    const int64_t dmax_geom = std::max<int64_t>(1, base.N / std::max<int64_t>(1, 2LL * base.r * K));
    std::vector<int> ds;
    if (in.n_chunks > 0) {
      ds.push_back(in.n_chunks);
    } else {
      for (int64_t d = 1; d <= std::min<int64_t>(dmax_geom, kMaxSearchChunks); ++d) ds.push_back((int)d);
    }
    for (int d : ds) {
      std::vector<int> kons;
      if (in.k_on > 0) {
        kons.push_back(std::min(in.k_on, K));
      } else if (in.method == SO2DR_METHOD_RESREU) {
        kons.push_back(1);
      } else {
        for (int k = 1; k <= std::min(K, 8); ++k)
          if (m.gupd[k - 1] > 0) kons.push_back(k);
      }
      for (int kon : kons) {
        so2dr_desc c = in;
        c.tb_depth = K;
        c.n_chunks = d;
        c.k_on = kon;
        Plan P;
        if (make_plan(c, &P) != SO2DR_OK) continue;
        const double t = predict_seconds(P, m, T);
        if (best < 0 || t < best * (1 - kMinGain)) {
          best = t;
          best_d = c;
          best_d.n_slots = in.n_slots > 0 ? in.n_slots : P.n_slots;
        }
      }
    }
  }
  if (best < 0) {
    set_error("no plan of the searched parameters fits the budget");
    return SO2DR_E_BUDGET;
  }
  *out = best_d;
  if (pred_ms) *pred_ms = 1e3 * best;
  set_error("");
  return SO2DR_OK;
}

}  // namespace so2dr
