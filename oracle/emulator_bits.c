/*
 * emulator_bits.c -- bit-level CPU model of the library's documented FP32
 * arithmetic, in C so that grids of tens of millions of cells can be checked
 * bit for bit.
 *
 * TEST INFRASTRUCTURE ONLY (like so2dr_oracle.c): nothing in the product
 * library links, includes or calls it, and it shares no code with the HIP
 * path.  It is written from the arithmetic the C interface documents, not
 * from the kernels:
 *   - every cell's new value is a chain of fused multiply-adds in FP32 that
 *     starts from +0 and runs over the stencil points in the order given
 *     (the lexicographic (dz, dy, dx) order of the weight array), with FP32
 *     weights:  acc = fmaf(w_k, ext(u, x + o_k), acc);
 *   - cells outside the grid come from the boundary rule (zero on a Dirichlet
 *     axis, wrapped on a periodic one), as in the Jacobi sweep of the paper's
 *     Sec. II-A;
 *   - after step t the field is rounded to the storage type (BF16 or FP16,
 *     round to nearest, ties to even) when round_flags is NULL or
 *     round_flags[t] != 0; otherwise it stays FP32.
 * fmaf is the C library's correctly rounded fused multiply-add (C11 7.12.13).
 * The Python model in emulator.py computes the same thing with an exact FMA
 * built from float64 products and TwoSum; the two are checked against each
 * other and against exact rational rounding in the tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { EMU_F32 = 0, EMU_BF16 = 2, EMU_F16 = 3 };

/* nearest-even bfloat16: keep the top 16 bits of the FP32 pattern, adding
 * half an ulp of the kept part (minus one when the kept part is even) */
static float round_bf16(float x) {
  uint32_t b;
  memcpy(&b, &x, 4);
  const uint32_t lsb = (b >> 16) & 1u;
  b = (b + 0x7fffu + lsb) & 0xffff0000u;
  memcpy(&x, &b, 4);
  return x;
}

/* nearest-even binary16: the quantum of a value of binade 2^E is 2^(E-10)
 * for normal halves (E >= -14) and 2^-24 below; rint() rounds to nearest
 * even in the default rounding mode; magnitudes that round to 2^16 or more
 * overflow to infinity (the largest half is 65504). */
static float round_f16(float x) {
  if (x == 0.0f || isnan(x) || isinf(x)) return x;
  const double d = x;
  int e;
  (void)frexp(d, &e);          /* 2^(e-1) <= |d| < 2^e */
  int q = (e - 1) - 10;
  if (q < -24) q = -24;
  double r = ldexp(rint(ldexp(d, -q)), q);
  if (fabs(r) >= 65536.0) r = copysign(INFINITY, d);
  return (float)r;
}

static float to_storage(float v, int storage) {
  if (storage == EMU_BF16) return round_bf16(v);
  if (storage == EMU_F16) return round_f16(v);
  return v;
}

/* index of coordinate c on an axis of length n under the boundary rule, or
 * -1 for a Dirichlet ghost */
static int64_t bc_index(int64_t c, int64_t n, int periodic) {
  if (c >= 0 && c < n) return c;
  if (!periodic) return -1;
  c %= n;
  return c < 0 ? c + n : c;
}

/* u_T from u0 (FP32 values, already representable in the storage type),
 * nx*ny*nz cells, x fastest.  offsets: npts (dz, dy, dx) triples in the
 * order of the sum; w: npts FP32 weights.  round_flags: NULL (round after
 * every step) or T+1 bytes, entry t for step t.  uT may alias u0. */
int emu_sweep(int64_t nx, int64_t ny, int64_t nz, const int *periodic, int npts, const int *off,
              const float *w, int T, int storage, const unsigned char *round_flags,
              const float *u0, float *uT) {
  if (nx < 1 || ny < 1 || nz < 1 || npts < 1 || !off || !w || T < 0 || !u0 || !uT) return -1;
  const int64_t n = nx * ny * nz;
  float *a = malloc(sizeof(float) * n), *b = malloc(sizeof(float) * n);
  if (!a || !b) { free(a); free(b); return -2; }
  memcpy(a, u0, sizeof(float) * n);
  const int px = periodic[0], py = periodic[1], pz = periodic[2];
  for (int t = 1; t <= T; ++t) {
    const int rnd = !round_flags || round_flags[t];
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
          float acc = 0.0f;
          for (int k = 0; k < npts; ++k) {
            const int *o = off + 3 * k;
            const int64_t X = bc_index(x + o[2], nx, px), Y = bc_index(y + o[1], ny, py),
                          Z = bc_index(z + o[0], nz, pz);
            const float v = (X < 0 || Y < 0 || Z < 0) ? 0.0f : a[(Z * ny + Y) * nx + X];
            acc = fmaf(w[k], v, acc);
          }
          b[(z * ny + y) * nx + x] = rnd ? to_storage(acc, storage) : acc;
        }
    float *s = a; a = b; b = s;
  }
  memcpy(uT, a, sizeof(float) * n);
  free(a); free(b);
  return 0;
}

/* The same values on the sub-box [b0, b1) (x, y, z; unreduced coordinates)
 * of a grid of nx*ny*nz cells, from a level-0 window covering the box dilated
 * by T*reach per axis (x fastest; values outside the grid already wrapped on
 * periodic axes, anything on Dirichlet axes).  Each step shrinks the window
 * by the reach: a cell of the box depends on nothing outside its dependency
 * cone, so the box comes out exactly as in a whole-grid sweep.  A cell
 * outside the grid on a Dirichlet axis is a ghost held at zero at every
 * level.  out: (b1 - b0) extents, x fastest. */
int emu_sweep_box_win(int64_t nx, int64_t ny, int64_t nz, const int *periodic, int npts,
                      const int *off, const float *w, int T, int storage,
                      const unsigned char *round_flags, const float *win, const int64_t *b0,
                      const int64_t *b1, float *out) {
  if (nx < 1 || ny < 1 || nz < 1 || npts < 1 || !off || !w || T < 0 || !win || !out) return -1;
  const int64_t n[3] = {nx, ny, nz};
  int64_t reach[3] = {0, 0, 0};
  for (int k = 0; k < npts; ++k)
    for (int q = 0; q < 3; ++q) {
      int64_t d = off[3 * k + 2 - q];
      if (d < 0) d = -d;
      if (d > reach[q]) reach[q] = d;
    }
  int64_t e[3], lo[3];
  for (int q = 0; q < 3; ++q) {
    if (b1[q] <= b0[q]) return -1;
    lo[q] = b0[q] - (int64_t)T * reach[q];
    e[q] = b1[q] - lo[q] + (int64_t)T * reach[q];
  }
  const int64_t cap = e[0] * e[1] * e[2];
  float *a = malloc(sizeof(float) * cap), *b = malloc(sizeof(float) * cap);
  if (!a || !b) { free(a); free(b); return -2; }
  memcpy(a, win, sizeof(float) * cap);
  /* level 0: ghosts of Dirichlet axes are zero */
  for (int64_t k = 0; k < e[2]; ++k)
    for (int64_t j = 0; j < e[1]; ++j)
      for (int64_t i = 0; i < e[0]; ++i) {
        const int64_t C[3] = {lo[0] + i, lo[1] + j, lo[2] + k};
        for (int q = 0; q < 3; ++q)
          if (!periodic[q] && (C[q] < 0 || C[q] >= n[q])) a[(k * e[1] + j) * e[0] + i] = 0.0f;
      }
  int64_t pe[3] = {e[0], e[1], e[2]}, plo[3] = {lo[0], lo[1], lo[2]};
  for (int t = 1; t <= T; ++t) {
    const int rnd = !round_flags || round_flags[t];
    int64_t ce[3], clo[3];
    for (int q = 0; q < 3; ++q) { clo[q] = plo[q] + reach[q]; ce[q] = pe[q] - 2 * reach[q]; }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ce[2]; ++k)
      for (int64_t j = 0; j < ce[1]; ++j)
        for (int64_t i = 0; i < ce[0]; ++i) {
          const int64_t C[3] = {clo[0] + i, clo[1] + j, clo[2] + k};
          int ghost = 0;
          for (int q = 0; q < 3; ++q)
            if (!periodic[q] && (C[q] < 0 || C[q] >= n[q])) ghost = 1;
          float acc = 0.0f;
          if (!ghost)
            for (int m = 0; m < npts; ++m) {
              const int *o = off + 3 * m;
              const int64_t pi = C[0] + o[2] - plo[0], pj = C[1] + o[1] - plo[1],
                            pk = C[2] + o[0] - plo[2];
              acc = fmaf(w[m], a[(pk * pe[1] + pj) * pe[0] + pi], acc);
            }
          b[(k * ce[1] + j) * ce[0] + i] = ghost ? 0.0f : rnd ? to_storage(acc, storage) : acc;
        }
    float *s = a; a = b; b = s;
    for (int q = 0; q < 3; ++q) { pe[q] = ce[q]; plo[q] = clo[q]; }
  }
  memcpy(out, a, sizeof(float) * pe[0] * pe[1] * pe[2]);
  free(a); free(b);
  return 0;
}
