/*
 * so2dr.h -- C interface of the out-of-core stencil library for MI355X.
 *
 * The library runs a time-stepped 2D/3D stencil sweep (paper Sec. II-A) on a
 * grid that lives in pinned host memory and may be far larger than the device
 * memory the caller grants it.  The grid is cut into chunks along its slowest
 * axis and streamed host -> HBM -> host (Sec. II-A, Fig. 1b).  Following
 * Algorithm 1 and Sec. IV, each chunk advances tb_depth steps per residency;
 * the round-start planes it shares with the next chunk are handed over in HBM
 * (the region-sharing buffer, Sec. II-B and Fig. 2) so they cross PCIe once;
 * and each chunk recomputes its shared overlap itself (Sec. IV-B, Fig. 4) so
 * its kernels can fuse k_on steps in LDS and registers.  The output of every
 * run equals the plain in-core Jacobi sweep; a plan with one chunk and
 * tb_depth = T is that in-core sweep, run by the same executor and kernels.
 *
 * Conventions shared by every call:
 *   - Grid layout: x fastest (contiguous), then y, then z.  A 3D grid is cut
 *     along z; a 2D grid (nz = 1) is cut along y.  Host arrays hold exactly
 *     nx*ny*nz elements of the storage type, no padding.
 *   - Every cell is updated every step; cells outside the grid come from the
 *     boundary rule of their axis (zero Dirichlet or periodic).  The cut axis
 *     must be zero Dirichlet.
 *   - Stencil weights: one double per stencil point, listed in lexicographic
 *     order of the (dz, dy, dx) offset triples (2D: (dy, dx)).  Star = the
 *     centre plus the axis points at distance 1..radius (Fig. 1a); box = the
 *     full (2r+1)^ndim cube (Table III).  Weight w multiplies the value at
 *     x + offset (a correlation).  Each cell's sum is formed in that same
 *     lexicographic order with fused multiply-adds, in FP32 for F32/BF16/F16
 *     storage (weights rounded to FP32) and in FP64 for F64 storage; BF16 and
 *     F16 results are rounded to nearest-even after every step.  The result of
 *     a run therefore does not depend on chunk count, tb_depth, k_on or slot
 *     count: only on the storage type.
 *   - Return codes: 0 on success, a negative SO2DR_E_* code otherwise; the
 *     thread-local message from so2dr_last_error() then says why.  No call
 *     throws or aborts.
 */
#ifndef SO2DR_H
#define SO2DR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SO2DR_OK 0
#define SO2DR_E_INVALID (-1)     /* malformed descriptor or argument */
#define SO2DR_E_BUDGET (-2)      /* no plan fits the device budget */
#define SO2DR_E_UNSUPPORTED (-3) /* stencil / dtype / depth not built */
#define SO2DR_E_NOT_PINNED (-4)  /* a host array is not pinned (page-locked) memory */
#define SO2DR_E_HIP (-5)         /* the HIP runtime reported an error */
#define SO2DR_E_UNBOUND (-6)     /* run before so2dr_plan_bind */

typedef enum { SO2DR_F32 = 0, SO2DR_F64 = 1, SO2DR_BF16 = 2, SO2DR_F16 = 3 } so2dr_dtype;
typedef enum { SO2DR_STAR = 0, SO2DR_BOX = 1 } so2dr_shape;
typedef enum { SO2DR_DIRICHLET0 = 0, SO2DR_PERIODIC = 1 } so2dr_bc;

/* Out-of-core method.  SO2DR (Sec. IV): round-start planes shared once per
 * round, overlap recomputed, k_on-step kernels.  RESREU (the paper's
 * comparison code, Sec. II-B / Fig. 2): intermediate results of every step
 * shared through the region-sharing buffer, so every kernel runs one step
 * and nothing is recomputed; kept for comparison. */
typedef enum { SO2DR_METHOD_SO2DR = 0, SO2DR_METHOD_RESREU = 1 } so2dr_method;

/* When BF16/F16 storage is rounded (FP32 and FP64 storage ignore this; no
 * counterpart in the paper, whose fields are FP32).
 *   SO2DR_ROUND_EVERY_STEP: after every time step, also between the levels a
 *     kernel fuses: the result depends on nothing but u0, the weights and T.
 *   SO2DR_ROUND_AT_STORE: fused levels keep FP32 sums in registers and LDS;
 *     only what a launch stores to HBM (every k_on steps, and at the end of
 *     each round of tb_depth steps) is rounded.  Fewer roundings, lower
 *     error; the result then depends on the launch schedule, and an
 *     out-of-core run equals the in-core run of the same k_on only when
 *     tb_depth is a multiple of k_on. */
typedef enum { SO2DR_ROUND_EVERY_STEP = 0, SO2DR_ROUND_AT_STORE = 1 } so2dr_rounding;

/* What carries the host <-> HBM copies (no counterpart in the paper, whose
 * copies are cudaMemcpyAsync).
 *   SO2DR_COPY_DMA: hipMemcpyAsync, the runtime's DMA engines.  Fastest for
 *     large copies (97 GB/s both directions together on MI355X); with many
 *     small copies enqueued at once its rate measured erratic, down to a
 *     third of that.
 *   SO2DR_COPY_KERNEL: a copy kernel of 64 workgroups per copy reads or
 *     writes the page-locked host array through its device mapping (about
 *     85 GB/s both directions together, independent of the copy size); the
 *     host array must be one page-locked allocation mapped into the device,
 *     else the run fails with E_NOT_PINNED.
 *   SO2DR_COPY_KERNEL_OUT: hipMemcpyAsync host -> HBM, copy kernels
 *     HBM -> host (same requirement on the host arrays).
 *   SO2DR_COPY_AUTO: KERNEL_OUT when the plan's largest chunk copy is
 *     below 512 MiB, a run of T steps queues more than 256 host copies
 *     (2 x chunks x rounds), the plan is not an adjoint plan and both host
 *     arrays are mapped; else DMA (thresholds measured on MI355X; 7-point
 *     2048x1024x1024 at 32 chunks: 88 GB/s KERNEL_OUT, 77 KERNEL, 42 DMA). */
typedef enum {
  SO2DR_COPY_AUTO = 0,
  SO2DR_COPY_DMA = 1,
  SO2DR_COPY_KERNEL = 2,
  SO2DR_COPY_KERNEL_OUT = 3
} so2dr_copy_engine;

/* Problem and run-time configuration: the variables of the paper's Table I
 * (dim, sz, r, d, S_tot, S_TB, N_strm, C_dmem) plus the stencil itself. */
typedef struct {
  int ndim;                   /* 2 or 3 */
  int64_t nx, ny, nz;         /* grid extents; nz must be 1 when ndim == 2 */
  int shape;                  /* so2dr_shape */
  int radius;                 /* stencil radius r >= 1 */
  const double *weights;      /* n_weights values, lexicographic (dz,dy,dx); copied */
  int n_weights;
  int bc[3];                  /* so2dr_bc for x, y, z; the cut axis must be DIRICHLET0 */
  int storage;                /* so2dr_dtype of host and HBM fields */
  int T;                      /* total time steps (S_tot) */
  int n_chunks;               /* d; 0 = choose the fewest that fit the budget */
  int tb_depth;               /* K = S_TB: steps per HBM residency; 0 = T */
  int k_on;                   /* steps fused per kernel launch; 0 = automatic */
  int n_slots;                /* chunks in flight (slot buffers): 0 = automatic (at most 3), else 1..4 */
  size_t device_budget_bytes; /* hard cap on the device memory the plan may use */
  int adjoint;                /* 1: also reserve what so2dr_adjoint_run needs */
  int method;                 /* so2dr_method: SO2DR_METHOD_SO2DR (default) or _RESREU */
  int rounding;               /* an so2dr_rounding value, for 16-bit storage; 0 = every step */
  int copy_engine;            /* an so2dr_copy_engine value; 0 = automatic */
} so2dr_desc;

/* What the planner chose (all sizes in bytes unless noted). */
typedef struct {
  int64_t n_axis;             /* length of the cut axis (planes) */
  int64_t plane_elems;        /* elements per plane */
  int n_chunks, tb_depth, k_on, n_slots, n_rounds;
  int max_chunk_planes;       /* planes owned by the largest chunk */
  int slot_planes;            /* planes in one slot buffer */
  int max_k_on;               /* deepest fused kernel built for this stencil */
  size_t workspace_bytes;     /* everything the plan uses; <= budget */
  size_t slot_bytes;          /* one slot: two ping-pong buffers (one when lean); an adjoint
                                 plan adds three buffers shared by all slots */
  size_t rs_bytes;            /* region-sharing buffer */
  size_t scratch_bytes;       /* reduction scratch (adjoint) */
  int lean;                   /* 1: one buffer per slot, kernels in shifted sub-blocks */
  int lean_block;             /* output planes per sub-block launch when lean */
  int method;                 /* so2dr_method of the plan */
  double redundant_fraction;  /* recomputed / useful cell updates */
  int64_t n_ops;              /* entries in the operation schedule */
  int rounding;               /* the so2dr_rounding value in effect: EVERY_STEP unless 16-bit storage */
  int copy_engine;            /* SO2DR_COPY_DMA, _KERNEL or _KERNEL_OUT: what runs use when the host
                                 arrays allow */
} so2dr_plan_info;

/* One entry of the schedule the executor runs (Algorithm 1, unrolled).
 * Plane ranges are half-open, in global plane indices of the cut axis. */
typedef enum {
  SO2DR_OP_H2D = 0,      /* host planes [z0,z1) -> slot buffer buf_out */
  SO2DR_OP_RS_READ = 1,  /* region-sharing buffer -> slot buffer buf_out planes [z0,z1) */
  SO2DR_OP_RS_WRITE = 2, /* slot buffer buf_in planes [z0,z1) -> region-sharing buffer */
  SO2DR_OP_KERNEL = 3,   /* levels steps: buf_in (valid [in_z0,in_z1)) -> buf_out [z0,z1);
                            in a lean plan buf_in == buf_out and the output lands below
                            every input plane a later operation still reads */
  SO2DR_OP_D2H = 4       /* slot buffer buf_in planes [z0,z1) -> host planes [z0,z1) */
} so2dr_op_kind;

typedef struct {
  int kind;               /* so2dr_op_kind */
  int round, chunk, slot;
  int64_t z0, z1;         /* planes written (H2D, RS_READ, KERNEL, D2H) or read (RS_WRITE) */
  int64_t in_z0, in_z1;   /* KERNEL: valid planes of the input level */
  int level_in;           /* KERNEL: time level (within the round) of the input */
  int levels;             /* KERNEL: steps fused in this launch */
  int buf_in, buf_out;    /* slot buffer index 0/1 (-1 when not used) */
  int64_t buf_z0;         /* global plane held at index 0 of the buffer read (or copied) */
  int64_t out_z0;         /* KERNEL: global plane held at index 0 of the buffer written */
  int64_t pool_off;       /* RS_READ/RS_WRITE: first plane used in the region-sharing buffer */
} so2dr_op;

/* Per-run measurements.  Times come from HIP events when timing is enabled
 * (so2dr_plan_set_timing), else they are 0 except wall_ms. */
typedef struct {
  double wall_ms;              /* first enqueue to last completion, host clock */
  double h2d_ms, d2h_ms, d2d_ms, kernel_ms;   /* summed event durations per category */
  uint64_t bytes_h2d, bytes_d2h, bytes_d2d;
  uint64_t kernel_launches;
  uint64_t cell_updates;       /* useful: nx*ny*nz*steps */
  uint64_t cell_updates_done;  /* including the redundant halo recomputation */
  uint64_t kernel_alg_bytes;   /* sum over launches of (input area + output area) * elem size */
  int rounds_done;
  /* the kernel figures split by fused depth: entry l-1 for launches of l
   * levels (kernel_ms_by_levels only with timing enabled) */
  double kernel_ms_by_levels[8];
  uint64_t launches_by_levels[8];
  uint64_t alg_bytes_by_levels[8];
} so2dr_stats;

/* Validate the descriptor and build the plan: chunk bounds, per-round depth
 * k' (Algorithm 1, rounds of tb_depth steps with the remainder last), the
 * per-launch fused depths, the shrinking compute areas of Sec. IV-B, slot
 * and region-sharing sizes, and the device-byte total, which must not exceed
 * device_budget_bytes.  Host-only: needs no GPU.  *out is owned by the caller
 * and released with so2dr_plan_destroy.  Errors: E_INVALID, E_BUDGET,
 * E_UNSUPPORTED. */
int so2dr_plan_create(const so2dr_desc *desc, struct so2dr_plan **out);

/* Release a plan (and the HIP events it created at bind time).  NULL is a no-op. */
void so2dr_plan_destroy(struct so2dr_plan *plan);

/* Planner outputs (host-only). */
int so2dr_plan_get_info(const struct so2dr_plan *plan, so2dr_plan_info *info);

/* Device bytes the caller must provide to so2dr_plan_bind (<= the budget). */
int so2dr_plan_workspace_bytes(const struct so2dr_plan *plan, size_t *bytes);

/* Copy the first n entries of the schedule into ops (host-only; n <= info.n_ops). */
int so2dr_plan_get_ops(const struct so2dr_plan *plan, so2dr_op *ops, int64_t n);

/* How the executor runs the schedule on n_streams streams (host-only; the
 * rules of so2dr_run and so2dr_run_steps, computed by the same code): op k
 * of so2dr_plan_get_ops is enqueued on stream index stream[k] (roles as in
 * so2dr_plan_bind) after waiting for the completion of the earlier ops
 * waits[k * SO2DR_MAX_WAITS + i] (-1 = none; ops on one stream also run in
 * list order).  The waits are what make the pipeline of Algorithm 1 safe:
 * slot reuse, copy-in before compute before copy-out, the region-sharing
 * buffer read before it is overwritten, and the in-place host array across
 * rounds.  n <= info.n_ops entries are written.  Errors: E_INVALID. */
#define SO2DR_MAX_WAITS 4
int so2dr_plan_get_deps(const struct so2dr_plan *plan, int n_streams, int32_t *stream,
                        int64_t *waits, int64_t n);

/* Attach device memory and streams.  dev_arena: device pointer to at least
 * so2dr_plan_workspace_bytes bytes, 256-byte aligned, owned by the caller and
 * not touched by anything else while a run is in flight.  streams: n_streams
 * HIP streams (hipStream_t as void*) at default priority, owned by the
 * caller.  Roles: streams[0] carries every host -> HBM copy in order,
 * streams[1] every HBM -> host copy, streams[2..n-1] the region-sharing
 * copies and kernels (chunk g on streams[2 + g % (n-2)]).  With n_streams == 2
 * the kernels share streams[0]; with 1 everything runs in order on it.
 * Recommended: 3 (one compute stream) or 4.  The plan keeps the pointers, not
 * the memory.  Errors: E_INVALID (null, misaligned or short arena), E_HIP. */
int so2dr_plan_bind(struct so2dr_plan *plan, void *dev_arena, size_t arena_bytes,
                    void *const *streams, int n_streams);

/* Testing aid for the failure path: the plan's next so2dr_run /
 * so2dr_run_steps stops with E_HIP after enqueuing n_ops operations of its
 * schedule (so2dr_plan_get_ops order), as if the HIP runtime had refused the
 * next one; -1 (the default) never.  One run only.  Errors: E_INVALID. */
int so2dr_plan_set_fail_after(struct so2dr_plan *plan, int64_t n_ops);

/* Enable (1) or disable (0) per-operation HIP event timing in so2dr_stats. */
int so2dr_plan_set_timing(struct so2dr_plan *plan, int enable);

/* Run the plan's T steps: host_u holds u_0 on entry and u_T on return, in
 * place (nx*ny*nz elements of the storage type, pinned).  Synchronous: the
 * array may be reused when the call returns, also after a failure (the work
 * already queued is drained first).  st may be NULL.
 * Errors: E_UNBOUND, E_NOT_PINNED, E_HIP (host contents then undefined;
 * st->rounds_done tells how many rounds completed). */
int so2dr_run(struct so2dr_plan *plan, void *host_u, so2dr_stats *st);

/* Bytes of the static device workspace so2dr_run_noalloc runs in. */
#define SO2DR_NOALLOC_MAX_BYTES ((size_t)128 << 20)

/* so2dr_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same executor and kernels, but the plan's workspace (slot buffers and the
 * region-sharing buffer) is a static device array of the library,
 * SO2DR_NOALLOC_MAX_BYTES bytes per GPU, held from the first call on a
 * device until the process ends; no hipMalloc, hipFree or other allocating
 * routine is called (the plan's HIP events are created on first use, as by
 * so2dr_run).  host_u: as for so2dr_run (pinned, u_0 in, u_T out, in place).
 * streams / n_streams: as for so2dr_plan_bind, on the current device, used
 * for this call only.  The plan need not be bound; a binding it has is left
 * as it was.  Nothing in the workspace has to start at zero: every byte a
 * kernel reads is written earlier in the same call.  Every call on one GPU
 * shares that GPU's array, so calls that overlap in time on one GPU race
 * (each returns only when its work is done, so calls from one thread never
 * overlap).  Errors: E_BUDGET (the plan's workspace exceeds
 * SO2DR_NOALLOC_MAX_BYTES), E_INVALID (null plan or stream), E_NOT_PINNED,
 * E_HIP (also when the array's device address cannot be obtained). */
int so2dr_run_noalloc(struct so2dr_plan *plan, void *host_u, void *const *streams, int n_streams,
                      so2dr_stats *st);

/* As so2dr_run but out of place and for `steps` steps (0 < steps <= T, same
 * chunking and depth): host_in is read-only, host_out receives u_steps.
 * host_in == host_out is the in-place run. */
int so2dr_run_steps(struct so2dr_plan *plan, const void *host_in, void *host_out, int steps,
                    so2dr_stats *st);

/* Adjoint of the whole sweep for L = 1/2 sum_x (u_T(x) - target(x))^2
 * (not in the paper; the transpose map of the same stencil, run backwards in
 * time with the same out-of-core machinery).  host_u0, host_target: inputs
 * (pinned, storage type F32 or F64).  host_grad_u0 receives dL/du_0; grad_w
 * receives n_weights doubles dL/dw (lexicographic order); *loss receives L.
 * The forward states at every ckpt_every-th step are kept in the caller's
 * pinned host buffers host_ckpt[0..n_ckpt-1] (each one field) and recomputed
 * in between.  n_ckpt must be >= ceil(T / ckpt_every).  Loss and weight
 * gradients are accumulated in FP64 on the GPU.
 * Errors: E_UNBOUND, E_NOT_PINNED, E_INVALID, E_UNSUPPORTED, E_HIP. */
int so2dr_adjoint_run(struct so2dr_plan *plan, const void *host_u0, const void *host_target,
                      void *host_grad_u0, double *grad_w, double *loss, int ckpt_every,
                      void *const *host_ckpt, int n_ckpt, so2dr_stats *st);

/* Page-locked host memory for the fields that runs read and write (host
 * memory management; not in the paper).  *ptr receives `bytes` bytes from
 * the HIP runtime's own page-locked allocator (default flags), 4096-byte
 * aligned and owned by the caller until so2dr_host_free; bytes == 0 gives
 * *ptr = NULL.  The allocation is mapped into the device, as copy kernels
 * (SO2DR_COPY_KERNEL) need, and its size is exactly `bytes`.
 * Errors: E_INVALID (null ptr), E_HIP (allocation failed; *ptr = NULL). */
int so2dr_host_alloc(size_t bytes, void **ptr);

/* Release memory from so2dr_host_alloc; NULL is a no-op.  Not while a run
 * that uses it is in flight.  Errors: E_HIP. */
int so2dr_host_free(void *ptr);

/* Machine figures for the cost model (no counterpart in the paper, which
 * leaves the automatic choice of chunk count and TB depth to future work,
 * Sec. IV-C and VII).  Rates in GB/s (1e9 bytes) and G cell-updates/s. */
typedef struct {
  double h2d_gbps, d2h_gbps;   /* pinned host copies, each direction alone */
  double duplex_gbps;          /* both directions at once, together */
  double d2d_gbps;             /* device-to-device copies */
  double launch_us;            /* fixed cost of one kernel launch */
  double gupd[8];              /* output cells x levels per second of a fused
                                  launch of 1..8 levels; 0 = not available */
  double kcopy_gbps;           /* both directions at once with copy kernels (COPY_KERNEL) */
  double kcopy_out_gbps;       /* both directions at once, DMA in and copy kernels out */
} so2dr_machine;

/* Fill *m with the library's built-in figures for this plan's stencil and
 * storage type (measured on MI355X: link rates of pinned copies, per-depth
 * update rates of the fused kernels).  Returns SO2DR_OK or E_INVALID. */
int so2dr_machine_default(const struct so2dr_plan *plan, so2dr_machine *m);

/* Predicted wall time in ms of `steps` steps (0 = the plan's T) of this plan:
 * its own operation schedule replayed through the executor's stream and
 * event rules with durations from *m (NULL = the built-in figures). */
int so2dr_plan_predict(const struct so2dr_plan *plan, const so2dr_machine *m, int steps,
                       double *ms);

/* Search the fields the caller left 0 -- tb_depth (K), n_chunks (d), k_on,
 * n_slots -- for the plan with the least predicted time that fits
 * device_budget_bytes, and write the completed descriptor to *out (the
 * weights pointer is copied, not the weights).  K is taken from a geometric
 * set up to T, d up to 32 and to the 2rK-planes-per-chunk limit; a
 * candidate replaces a cheaper-looking earlier one (fewer chunks, levels or
 * shallower rounds) only when predicted more than 1 % faster.  *ms (may be
 * NULL) receives the predicted time.  Returns SO2DR_OK, the descriptor's
 * validation error, or E_BUDGET when no candidate fits. */
int so2dr_plan_suggest(const so2dr_desc *desc, const so2dr_machine *m, so2dr_desc *out,
                       double *ms);

/* Time one fused-step launch of the plan's stencil and storage type on
 * device memory the caller owns (measurement; the rates behind the cost
 * model's per-depth figures and the kernels' roofline positions).  dev_in,
 * dev_out: device buffers of in_planes planes each (plane = nx * ny elements
 * of the storage type); dev_in is read as an interior chunk of the cut axis
 * (the planes in its middle), and the launch advances it by `levels` steps
 * into planes [levels * radius, in_planes - levels * radius) of dev_out.
 * levels == 0 times the library's device copy kernel over the in_planes
 * planes instead.  One untimed launch, then `reps` launches back to back on
 * `stream` between two HIP events; *ms receives the mean time per launch.
 * Errors: E_INVALID (levels outside [0, max_k_on], in_planes <= 2 levels r
 * or beyond the cut axis, null pointers, reps < 1), E_UNSUPPORTED, E_HIP. */
int so2dr_kernel_bench(const struct so2dr_plan *plan, int levels, void *dev_in, void *dev_out,
                       int64_t in_planes, int reps, void *stream, double *ms);

/* Host-link rates with the copies the executor issues (measurement): bytes
 * from pinned host_a to device dev_a on stream_in (host -> HBM), from dev_b
 * to pinned host_b on stream_out (HBM -> host), each as `pieces`
 * hipMemcpyAsync calls of bytes / pieces queued back to back (the two
 * directions interleaved), each direction alone and both at once;
 * gbps[0..2] receive the best of `reps` passes (after one warm-up pass) in
 * GB/s (1e9 bytes; both at once: the two directions' bytes together).  The
 * caller owns all four buffers (bytes each) and the two distinct streams.
 * Errors: E_INVALID (also bytes not a multiple of pieces), E_NOT_PINNED,
 * E_HIP. */
int so2dr_link_probe(void *host_a, void *host_b, void *dev_a, void *dev_b, size_t bytes, int pieces,
                     void *stream_in, void *stream_out, int reps, double *gbps);

/* Message describing the last error on this thread ("" if none). */
const char *so2dr_last_error(void);

/* Library version string. */
const char *so2dr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SO2DR_H */
