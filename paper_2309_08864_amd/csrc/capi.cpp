// capi.cpp -- the extern "C" boundary.  Every entry point validates its
// arguments, catches every C++ exception and reports failures through a
// return code plus a thread-local message.
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "plan.hpp"

struct so2dr_plan {
  so2dr::Plan p;
};

namespace so2dr {
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
int bind_plan(Plan &P, void *arena, size_t bytes, void *const *streams, int n_streams);
int execute(Plan &P, const void *host_in, void *host_out, int steps, so2dr_stats *st);
int adjoint_run(Plan &P, const void *u0, const void *target, void *grad_u0, double *grad_w,
                double *loss, int ckpt_every, void *const *ckpt, int n_ckpt, so2dr_stats *st);
void default_machine(const Plan &P, so2dr_machine *m);
double predict_seconds(const Plan &P, const so2dr_machine &m, int steps);
int suggest(const so2dr_desc &in, const so2dr_machine *mp, so2dr_desc *out, double *pred_ms);
int kernel_bench(const Plan &P, int levels, void *dev_in, void *dev_out, int64_t in_planes, int reps,
                 hipStream_t s, double *ms);
int link_probe(void *host_a, void *host_b, void *dev_a, void *dev_b, size_t bytes, int pieces,
               hipStream_t s_in, hipStream_t s_out, int reps, double *gbps);
}  // namespace so2dr

using so2dr::set_error;

// Device workspace of so2dr_run_noalloc: one array per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address comes from hipGetSymbolAddress, asked
// once per device (with that device current) and kept in g_scratch_dev.
static __device__ __align__(256) unsigned char scratch[SO2DR_NOALLOC_MAX_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, or null with the error set.
void *scratch_on_current_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error(std::string("hipGetDevice: ") + (e != hipSuccess ? hipGetErrorString(e) : "device index out of range"));
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") +
                (e != hipSuccess ? hipGetErrorString(e) : "null address"));
      return nullptr;
    }
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}
}  // namespace

#define GUARD_BEGIN try {
#define GUARD_END                                            \
  }                                                          \
  catch (const std::bad_alloc &) {                           \
    set_error("host allocation failed");                     \
    return SO2DR_E_INVALID;                                  \
  }                                                          \
  catch (const std::exception &e) {                          \
    set_error(std::string("internal error: ") + e.what());   \
    return SO2DR_E_INVALID;                                  \
  }                                                          \
  catch (...) {                                              \
    set_error("internal error");                             \
    return SO2DR_E_INVALID;                                  \
  }

extern "C" {

int so2dr_plan_create(const so2dr_desc *desc, so2dr_plan **out) {
  GUARD_BEGIN
  if (!desc || !out) {
    set_error("null descriptor or output pointer");
    return SO2DR_E_INVALID;
  }
  *out = nullptr;
  so2dr_plan *h = new so2dr_plan();
  const int rc = so2dr::make_plan(*desc, &h->p);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  set_error("");
  return SO2DR_OK;
  GUARD_END
}

void so2dr_plan_destroy(so2dr_plan *plan) {
  try {
    delete plan;
  } catch (...) {
  }
}

int so2dr_plan_get_info(const so2dr_plan *plan, so2dr_plan_info *info) {
  GUARD_BEGIN
  if (!plan || !info) {
    set_error("null plan or info");
    return SO2DR_E_INVALID;
  }
  const so2dr::Plan &P = plan->p;
  std::memset(info, 0, sizeof(*info));
  info->n_axis = P.N;
  info->plane_elems = P.plane;
  info->n_chunks = P.d;
  info->tb_depth = P.K;
  info->k_on = P.k_on;
  info->n_slots = P.n_slots;
  info->n_rounds = so2dr::n_rounds_for(P, P.T);
  int64_t mx = 0;
  for (int i = 0; i < P.d; ++i) mx = std::max<int64_t>(mx, P.bnd[i + 1] - P.bnd[i]);
  info->max_chunk_planes = (int)mx;
  info->slot_planes = (int)P.slot_planes;
  info->max_k_on = P.max_k_on;
  info->workspace_bytes = P.workspace;
  info->slot_bytes = (size_t)P.bufs_per_slot * P.buf_bytes;
  info->rs_bytes = P.rs_bytes;
  info->scratch_bytes = P.scratch_bytes;
  info->lean = P.lean ? 1 : 0;
  info->lean_block = P.lean_block;
  info->method = P.resreu ? SO2DR_METHOD_RESREU : SO2DR_METHOD_SO2DR;
  int64_t computed = 0;
  auto ops = so2dr::build_ops(P, P.T, &computed);
  info->n_ops = (int64_t)ops.size();
  const double useful = (double)P.N * (double)P.T;
  info->redundant_fraction = useful > 0 ? (double)computed / useful - 1.0 : 0.0;
  info->rounding = P.ras ? SO2DR_ROUND_AT_STORE : SO2DR_ROUND_EVERY_STEP;
  info->copy_engine = P.copy_engine;
  return SO2DR_OK;
  GUARD_END
}

int so2dr_plan_workspace_bytes(const so2dr_plan *plan, size_t *bytes) {
  GUARD_BEGIN
  if (!plan || !bytes) {
    set_error("null plan or output");
    return SO2DR_E_INVALID;
  }
  *bytes = plan->p.workspace;
  return SO2DR_OK;
  GUARD_END
}

int so2dr_plan_get_ops(const so2dr_plan *plan, so2dr_op *ops, int64_t n) {
  GUARD_BEGIN
  if (!plan || (!ops && n > 0) || n < 0) {
    set_error("null plan or ops");
    return SO2DR_E_INVALID;
  }
  auto all = so2dr::build_ops(plan->p, plan->p.T, nullptr);
  if (n > (int64_t)all.size()) {
    set_error("n exceeds the schedule length");
    return SO2DR_E_INVALID;
  }
  if (n > 0) std::memcpy(ops, all.data(), sizeof(so2dr_op) * (size_t)n);
  return SO2DR_OK;
  GUARD_END
}

int so2dr_plan_get_deps(const so2dr_plan *plan, int n_streams, int32_t *stream, int64_t *waits,
                        int64_t n) {
  GUARD_BEGIN
  if (!plan || n < 0 || (n > 0 && (!stream || !waits)) || n_streams < 1) {
    set_error("null plan or output, negative n, or no stream");
    return SO2DR_E_INVALID;
  }
  auto all = so2dr::build_ops(plan->p, plan->p.T, nullptr);
  if (n > (int64_t)all.size()) {
    set_error("n exceeds the schedule length");
    return SO2DR_E_INVALID;
  }
  std::vector<int> strm;
  std::vector<int64_t> w;
  so2dr::schedule_deps(plan->p, all, n_streams, &strm, &w);
  for (int64_t k = 0; k < n; ++k) {
    stream[k] = strm[(size_t)k];
    for (int i = 0; i < SO2DR_MAX_WAITS; ++i) waits[k * SO2DR_MAX_WAITS + i] = w[(size_t)k * so2dr::kMaxWaits + i];
  }
  return SO2DR_OK;
  GUARD_END
}

int so2dr_machine_default(const so2dr_plan *plan, so2dr_machine *m) {
  GUARD_BEGIN
  if (!plan || !m) {
    set_error("null plan or machine");
    return SO2DR_E_INVALID;
  }
  so2dr::default_machine(plan->p, m);
  return SO2DR_OK;
  GUARD_END
}

int so2dr_plan_predict(const so2dr_plan *plan, const so2dr_machine *m, int steps, double *ms) {
  GUARD_BEGIN
  if (!plan || !ms || steps < 0) {
    set_error("null plan or output, or negative steps");
    return SO2DR_E_INVALID;
  }
  so2dr_machine dm;
  if (!m) so2dr::default_machine(plan->p, &dm);
  *ms = 1e3 * so2dr::predict_seconds(plan->p, m ? *m : dm, steps ? steps : plan->p.T);
  return SO2DR_OK;
  GUARD_END
}

int so2dr_plan_suggest(const so2dr_desc *desc, const so2dr_machine *m, so2dr_desc *out, double *ms) {
  GUARD_BEGIN
  if (!desc || !out) {
    set_error("null descriptor or output");
    return SO2DR_E_INVALID;
  }
  return so2dr::suggest(*desc, m, out, ms);
  GUARD_END
}

int so2dr_plan_bind(so2dr_plan *plan, void *dev_arena, size_t arena_bytes, void *const *streams,
                    int n_streams) {
  GUARD_BEGIN
  if (!plan) {
    set_error("null plan");
    return SO2DR_E_INVALID;
  }
  return so2dr::bind_plan(plan->p, dev_arena, arena_bytes, streams, n_streams);
  GUARD_END
}

int so2dr_plan_set_timing(so2dr_plan *plan, int enable) {
  GUARD_BEGIN
  if (!plan) {
    set_error("null plan");
    return SO2DR_E_INVALID;
  }
  plan->p.timing = enable != 0;
  return SO2DR_OK;
  GUARD_END
}

int so2dr_plan_set_fail_after(so2dr_plan *plan, int64_t n_ops) {
  GUARD_BEGIN
  if (!plan || n_ops < -1) {
    set_error("null plan or n_ops < -1");
    return SO2DR_E_INVALID;
  }
  plan->p.fail_after_ops = n_ops;
  return SO2DR_OK;
  GUARD_END
}

int so2dr_run(so2dr_plan *plan, void *host_u, so2dr_stats *st) {
  GUARD_BEGIN
  if (!plan) {
    set_error("null plan");
    return SO2DR_E_INVALID;
  }
  return so2dr::execute(plan->p, host_u, host_u, plan->p.T, st);
  GUARD_END
}

int so2dr_run_noalloc(so2dr_plan *plan, void *host_u, void *const *streams, int n_streams,
                      so2dr_stats *st) {
  GUARD_BEGIN
  if (!plan) {
    set_error("null plan");
    return SO2DR_E_INVALID;
  }
  so2dr::Plan &P = plan->p;
  if (P.workspace > SO2DR_NOALLOC_MAX_BYTES) {
    set_error("plan workspace of " + std::to_string(P.workspace) +
              " bytes exceeds the static workspace of so2dr_run_noalloc (" +
              std::to_string((size_t)SO2DR_NOALLOC_MAX_BYTES) + " bytes)");
    return SO2DR_E_BUDGET;
  }
  if (!streams || n_streams < 1) {
    set_error("at least one stream is needed");
    return SO2DR_E_INVALID;
  }
  for (int i = 0; i < n_streams; ++i)
    if (!streams[i]) {
      set_error("null stream");
      return SO2DR_E_INVALID;
    }
  char *ws = static_cast<char *>(scratch_on_current_device());
  if (!ws) return SO2DR_E_HIP;
  // run on the static workspace, then give the plan back whatever binding
  // it had (so2dr_run keeps working on the caller's arena)
  char *old_arena = P.arena;
  const size_t old_bytes = P.arena_bytes;
  std::vector<hipStream_t> old_streams = P.streams;
  const bool old_bound = P.bound;
  P.arena = ws;
  P.arena_bytes = SO2DR_NOALLOC_MAX_BYTES;
  P.streams.clear();
  for (int i = 0; i < n_streams; ++i) P.streams.push_back(static_cast<hipStream_t>(streams[i]));
  P.bound = true;
  const int rc = so2dr::execute(P, host_u, host_u, P.T, st);
  P.arena = old_arena;
  P.arena_bytes = old_bytes;
  P.streams.swap(old_streams);
  P.bound = old_bound;
  return rc;
  GUARD_END
}

int so2dr_run_steps(so2dr_plan *plan, const void *host_in, void *host_out, int steps,
                    so2dr_stats *st) {
  GUARD_BEGIN
  if (!plan) {
    set_error("null plan");
    return SO2DR_E_INVALID;
  }
  if (steps < 1) {
    set_error("steps must be >= 1");
    return SO2DR_E_INVALID;
  }
  return so2dr::execute(plan->p, host_in, host_out, steps, st);
  GUARD_END
}

int so2dr_adjoint_run(so2dr_plan *plan, const void *host_u0, const void *host_target,
                      void *host_grad_u0, double *grad_w, double *loss, int ckpt_every,
                      void *const *host_ckpt, int n_ckpt, so2dr_stats *st) {
  GUARD_BEGIN
  if (!plan) {
    set_error("null plan");
    return SO2DR_E_INVALID;
  }
  return so2dr::adjoint_run(plan->p, host_u0, host_target, host_grad_u0, grad_w, loss,
                            ckpt_every, host_ckpt, n_ckpt, st);
  GUARD_END
}

int so2dr_kernel_bench(const so2dr_plan *plan, int levels, void *dev_in, void *dev_out,
                       int64_t in_planes, int reps, void *stream, double *ms) {
  GUARD_BEGIN
  if (!plan) {
    set_error("null plan");
    return SO2DR_E_INVALID;
  }
  return so2dr::kernel_bench(plan->p, levels, dev_in, dev_out, in_planes, reps,
                             static_cast<hipStream_t>(stream), ms);
  GUARD_END
}

int so2dr_link_probe(void *host_a, void *host_b, void *dev_a, void *dev_b, size_t bytes, int pieces,
                     void *stream_in, void *stream_out, int reps, double *gbps) {
  GUARD_BEGIN
  return so2dr::link_probe(host_a, host_b, dev_a, dev_b, bytes, pieces, static_cast<hipStream_t>(stream_in),
                           static_cast<hipStream_t>(stream_out), reps, gbps);
  GUARD_END
}

int so2dr_host_alloc(size_t bytes, void **ptr) {
  if (!ptr) {
    set_error("null output pointer");
    return SO2DR_E_INVALID;
  }
  *ptr = nullptr;
  if (bytes == 0) return SO2DR_OK;
  void *p = nullptr;
  const hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    set_error(std::string("hipHostMalloc: ") + hipGetErrorString(e));
    return SO2DR_E_HIP;
  }
  *ptr = p;
  set_error("");
  return SO2DR_OK;
}

int so2dr_host_free(void *ptr) {
  if (!ptr) return SO2DR_OK;
  const hipError_t e = hipHostFree(ptr);
  if (e != hipSuccess) {
    set_error(std::string("hipHostFree: ") + hipGetErrorString(e));
    return SO2DR_E_HIP;
  }
  return SO2DR_OK;
}

const char *so2dr_last_error(void) { return so2dr::g_err.c_str(); }

const char *so2dr_version(void) { return "so2dr-mi355x 0.1 (gfx950)"; }

}  // extern "C"
