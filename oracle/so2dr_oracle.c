/*
 * so2dr_oracle.c -- plain FP64 CPU reference for the time-stepped stencil sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no header, table or helper with the HIP path.
 *
 * What it computes (paper, Sec. II-A and Fig. 1a; Sec. IV-B for why the
 * out-of-core method must reproduce it exactly):
 *   u_{t+1}(x) = sum_k w_k * ext(u_t, x + o_k)        for every cell x,
 * a Jacobi (two-array) update, written as a correlation: weight w_k multiplies
 * the value at x + o_k.  ext() supplies the boundary: zero outside the grid on
 * a Dirichlet axis, index modulo n on a periodic axis.  The out-of-core
 * chunked sweep with region sharing and redundant halo computation reaches
 * this same result, which is why the oracle is the in-core definition and
 * nothing else.
 *
 * The adjoint (reverse-mode gradient of L = 1/2 ||u_T - y||^2) follows from
 * the chain rule applied to the same linear map:
 *   lambda_T = u_T - y
 *   lambda_t(x) = sum_k w_k * ext(lambda_{t+1}, x - o_k)       (transpose)
 *   dL/dw_k     = sum_t sum_x lambda_{t+1}(x) * ext(u_t, x + o_k)
 *   dL/du_0     = lambda_0
 * The paper has no adjoint; this is the plain mathematics of the map above.
 *
 * Grid layout: nx*ny*nz doubles, x fastest.  A 2D grid is nz == 1 with every
 * offset's dz == 0.  Offsets are given by the caller as (dz, dy, dx) triples;
 * the sum runs over them in the order given.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n[3];     /* nx, ny, nz */
  int periodic[3];  /* per axis x, y, z: 1 = periodic, 0 = zero Dirichlet */
  int npts;
  const int *off;   /* npts * 3 : dz, dy, dx */
  const double *w;  /* npts */
} grid_t;

/* Value of field f at (x, y, z) under the boundary rule; coordinates may lie
 * outside the grid. */
static double ext(const grid_t *g, const double *f, int64_t x, int64_t y, int64_t z) {
  int64_t c[3] = {x, y, z};
  for (int a = 0; a < 3; ++a) {
    if (c[a] < 0 || c[a] >= g->n[a]) {
      if (!g->periodic[a]) return 0.0;
      c[a] %= g->n[a];
      if (c[a] < 0) c[a] += g->n[a];
    }
  }
  return f[(c[2] * g->n[1] + c[1]) * g->n[0] + c[0]];
}

/* One forward step: dst(x) = sum_k w_k ext(src, x + o_k). sign = -1 gives the
 * transpose step dst(x) = sum_k w_k ext(src, x - o_k). */
static void step(const grid_t *g, const double *src, double *dst, int sign) {
  const int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for schedule(static)
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        double acc = 0.0;
        for (int k = 0; k < g->npts; ++k) {
          const int *o = g->off + 3 * k;
          acc += g->w[k] * ext(g, src, x + sign * o[2], y + sign * o[1], z + sign * o[0]);
        }
        dst[(z * ny + y) * nx + x] = acc;
      }
}

static int setup(grid_t *g, int64_t nx, int64_t ny, int64_t nz, const int *periodic,
                 int npts, const int *off, const double *w) {
  if (nx < 1 || ny < 1 || nz < 1 || npts < 1 || !off || !w) return -1;
  g->n[0] = nx; g->n[1] = ny; g->n[2] = nz;
  for (int a = 0; a < 3; ++a) g->periodic[a] = periodic ? periodic[a] : 0;
  g->npts = npts; g->off = off; g->w = w;
  return 0;
}

/* u_T from u_0 by T forward steps.  u0 and uT may be the same array. */
int oracle_sweep(int64_t nx, int64_t ny, int64_t nz, const int *periodic,
                 int npts, const int *off, const double *w, int T,
                 const double *u0, double *uT) {
  grid_t g;
  if (setup(&g, nx, ny, nz, periodic, npts, off, w) || T < 0) return -1;
  const int64_t n = nx * ny * nz;
  double *a = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n);
  if (!a || !b) { free(a); free(b); return -2; }
  memcpy(a, u0, sizeof(double) * n);
  for (int t = 0; t < T; ++t) { step(&g, a, b, +1); double *s = a; a = b; b = s; }
  memcpy(uT, a, sizeof(double) * n);
  free(a); free(b);
  return 0;
}

/* One transpose step (the adjoint of one forward step). */
int oracle_transpose_step(int64_t nx, int64_t ny, int64_t nz, const int *periodic,
                          int npts, const int *off, const double *w,
                          const double *src, double *dst) {
  grid_t g;
  if (setup(&g, nx, ny, nz, periodic, npts, off, w) || src == dst) return -1;
  step(&g, src, dst, -1);
  return 0;
}

/* Loss, gradient w.r.t. u_0 and w.r.t. every weight, for
 * L = 1/2 sum_x (u_T(x) - y(x))^2.  States are kept every `ckpt` steps and the
 * ones in between are recomputed segment by segment (ckpt <= 0: every step is
 * kept).  uT_out may be NULL. */
int oracle_adjoint(int64_t nx, int64_t ny, int64_t nz, const int *periodic,
                   int npts, const int *off, const double *w, int T,
                   const double *u0, const double *target, int ckpt,
                   double *loss, double *grad_u0, double *grad_w, double *uT_out) {
  grid_t g;
  if (setup(&g, nx, ny, nz, periodic, npts, off, w) || T < 0) return -1;
  if (ckpt <= 0 || ckpt > T) ckpt = T > 0 ? T : 1;
  const int64_t n = nx * ny * nz;
  const int nseg = (T + ckpt - 1) / ckpt;
  /* saved[j] = u_{j*ckpt}; seg[m] = u_{j*ckpt + m} inside the current segment */
  double *saved = malloc(sizeof(double) * n * (size_t)(nseg > 0 ? nseg : 1));
  double *seg = malloc(sizeof(double) * n * (size_t)ckpt);
  double *cur = malloc(sizeof(double) * n), *nxt = malloc(sizeof(double) * n);
  double *lam = malloc(sizeof(double) * n), *lam2 = malloc(sizeof(double) * n);
  double *part = malloc(sizeof(double) * nz);
  if (!saved || !seg || !cur || !nxt || !lam || !lam2 || !part) {
    free(saved); free(seg); free(cur); free(nxt); free(lam); free(lam2); free(part); return -2;
  }
  /* forward pass, keeping checkpoints */
  memcpy(cur, u0, sizeof(double) * n);
  for (int t = 0; t < T; ++t) {
    if (t % ckpt == 0) memcpy(saved + (size_t)(t / ckpt) * n, cur, sizeof(double) * n);
    step(&g, cur, nxt, +1);
    double *s = cur; cur = nxt; nxt = s;
  }
  if (uT_out) memcpy(uT_out, cur, sizeof(double) * n);
  /* loss and lambda_T */
  double l = 0.0;
  for (int64_t i = 0; i < n; ++i) { lam[i] = cur[i] - target[i]; l += 0.5 * lam[i] * lam[i]; }
  *loss = l;
  for (int k = 0; k < npts; ++k) grad_w[k] = 0.0;
  /* reverse pass, one segment at a time */
  for (int j = nseg - 1; j >= 0; --j) {
    const int t0 = j * ckpt, t1 = (t0 + ckpt < T) ? t0 + ckpt : T;
    memcpy(seg, saved + (size_t)j * n, sizeof(double) * n);
    for (int t = t0 + 1; t < t1; ++t)
      step(&g, seg + (size_t)(t - 1 - t0) * n, seg + (size_t)(t - t0) * n, +1);
    for (int t = t1 - 1; t >= t0; --t) {
      const double *ut = seg + (size_t)(t - t0) * n;   /* u_t; lam holds lambda_{t+1} */
      for (int k = 0; k < npts; ++k) {
        const int *o = off + 3 * k;
        /* per-plane partial sums, then added in plane order: the result does
         * not depend on the thread count */
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < nz; ++z) {
          double s = 0.0;
          for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x)
              s += lam[(z * ny + y) * nx + x] * ext(&g, ut, x + o[2], y + o[1], z + o[0]);
          part[z] = s;
        }
        double s = 0.0;
        for (int64_t z = 0; z < nz; ++z) s += part[z];
        grad_w[k] += s;
      }
      step(&g, lam, lam2, -1);
      double *q = lam; lam = lam2; lam2 = q;
    }
  }
  memcpy(grad_u0, lam, sizeof(double) * n);
  free(saved); free(seg); free(cur); free(nxt); free(lam); free(lam2); free(part);
  return 0;
}

/* u_T on the sub-box [b0, b1) (per axis x, y, z) only, computed from the part
 * of u_0 that can reach it: the box dilated by T*reach, where reach is the
 * largest |offset| along each axis.  Level t is formed on the box dilated by
 * (T - t)*reach.  Coordinates are kept unreduced: on a periodic axis a value
 * at an outside coordinate equals the wrapped cell's, on a Dirichlet axis a
 * cell outside the grid is the zero boundary at every level.  Used to check
 * grids too large for the full sweep on a few sampled boxes.
 * out: (b1-b0) extents, x fastest. */
static int sweep_box_impl(int64_t nx, int64_t ny, int64_t nz, const int *periodic,
                          int npts, const int *off, const double *w, int T,
                          const double *u0, const double *win, const int64_t *b0,
                          const int64_t *b1, double *out) {
  grid_t g;
  if (setup(&g, nx, ny, nz, periodic, npts, off, w) || T < 0) return -1;
  int64_t reach[3] = {0, 0, 0};
  for (int k = 0; k < npts; ++k)
    for (int a = 0; a < 3; ++a) {
      int64_t d = off[3 * k + 2 - a];
      if (d < 0) d = -d;
      if (d > reach[a]) reach[a] = d;
    }
  for (int a = 0; a < 3; ++a) if (b1[a] <= b0[a]) return -1;
  /* largest (level 0) extents */
  int64_t e[3], lo[3];
  for (int a = 0; a < 3; ++a) { lo[a] = b0[a] - (int64_t)T * reach[a]; e[a] = b1[a] - lo[a] + (int64_t)T * reach[a]; }
  const int64_t cap = e[0] * e[1] * e[2];
  double *a = malloc(sizeof(double) * cap), *b = malloc(sizeof(double) * cap);
  if (!a || !b) { free(a); free(b); return -2; }
  /* level 0 over the full window: from u0 under the boundary rule, or, when
   * u0 is NULL, from the caller's window (already extended, same extents) */
  for (int64_t k = 0; k < e[2]; ++k)
    for (int64_t j = 0; j < e[1]; ++j)
      for (int64_t i = 0; i < e[0]; ++i)
        a[(k * e[1] + j) * e[0] + i] =
            u0 ? ext(&g, u0, lo[0] + i, lo[1] + j, lo[2] + k) : win[(k * e[1] + j) * e[0] + i];
  int64_t pe[3] = {e[0], e[1], e[2]}, plo[3] = {lo[0], lo[1], lo[2]};
  for (int t = 1; t <= T; ++t) {
    int64_t ce[3], clo[3];
    for (int q = 0; q < 3; ++q) { clo[q] = plo[q] + reach[q]; ce[q] = pe[q] - 2 * reach[q]; }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ce[2]; ++k)
      for (int64_t j = 0; j < ce[1]; ++j)
        for (int64_t i = 0; i < ce[0]; ++i) {
          const int64_t X = clo[0] + i, Y = clo[1] + j, Z = clo[2] + k;
          const int64_t C[3] = {X, Y, Z};
          int outside = 0;
          for (int q = 0; q < 3; ++q)
            if (!g.periodic[q] && (C[q] < 0 || C[q] >= g.n[q])) outside = 1;
          double acc = 0.0;
          if (!outside)
            for (int m = 0; m < npts; ++m) {
              const int *o = off + 3 * m;
              const int64_t pi = X + o[2] - plo[0], pj = Y + o[1] - plo[1], pk = Z + o[0] - plo[2];
              acc += w[m] * a[(pk * pe[1] + pj) * pe[0] + pi];
            }
          b[(k * ce[1] + j) * ce[0] + i] = acc;
        }
    double *s = a; a = b; b = s;
    for (int q = 0; q < 3; ++q) { pe[q] = ce[q]; plo[q] = clo[q]; }
  }
  memcpy(out, a, sizeof(double) * pe[0] * pe[1] * pe[2]);
  free(a); free(b);
  return 0;
}

int oracle_sweep_box(int64_t nx, int64_t ny, int64_t nz, const int *periodic,
                     int npts, const int *off, const double *w, int T,
                     const double *u0, const int64_t *b0, const int64_t *b1,
                     double *out) {
  if (!u0) return -1;
  return sweep_box_impl(nx, ny, nz, periodic, npts, off, w, T, u0, NULL, b0, b1, out);
}

/* As oracle_sweep_box, with level 0 given directly as the window: the box
 * dilated by T*reach per axis, x fastest, in unreduced coordinates (values
 * outside the grid already wrapped or zeroed by the boundary rule). */
int oracle_sweep_box_win(int64_t nx, int64_t ny, int64_t nz, const int *periodic,
                         int npts, const int *off, const double *w, int T,
                         const double *win, const int64_t *b0, const int64_t *b1,
                         double *out) {
  if (!win) return -1;
  return sweep_box_impl(nx, ny, nz, periodic, npts, off, w, T, NULL, win, b0, b1, out);
}
