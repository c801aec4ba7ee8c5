// tb_kernel.hpp -- the k_on-step temporal-blocking stencil kernel for gfx950.
//
// One launch advances a chunk's compute area by KL time levels (paper
// Sec. III: on-chip data reuse lets one kernel proceed several steps;
// Algorithm 1 applies k_on-step kernels and one remainder kernel per round).
// The compute area of each level is the one the planner hands over: the
// shrinking parallelogram of Sec. IV-B, so every plane a valid output needs
// is either valid input or a zero Dirichlet ghost outside the grid.
//
// Work decomposition (CDNA4-first, not a port of the paper's AN5D kernels):
//   * a workgroup of 256 lanes (4 wave64) owns one xy tile of TX x TY input
//     cells, overlapped with its neighbours by KL*R cells per side, and one
//     segment of output planes along the cut axis;
//   * it marches that segment plane by plane.  Each march step loads one new
//     input plane (prefetched one step ahead), publishes the newest plane of
//     every level 0..KL-1 into LDS (double-buffered, so one barrier per step),
//     and lets every level 1..KL consume the plane its predecessor published;
//   * each level keeps, per owned cell, 2R+1 partial sums in registers: the
//     outputs that the consumed plane contributes to.  A plane arriving at
//     offset dz adds its (dy, dx) footprint to the sum of output plane p - dz.
//     Planes arrive in increasing order, so every output's fused
//     multiply-add chain runs in lexicographic (dz, dy, dx) order -- the order
//     of the weight array -- whatever the tiling, segmenting or chunking.
//     That makes out-of-core and in-core results bit-identical;
//   * the xy halo of the tile shrinks by R per level (redundant tile-edge
//     computation, the on-chip counterpart of the paper's off-chip one);
//   * cells outside the grid on a Dirichlet axis are ghosts held at zero at
//     every level; on a periodic axis the tile reads wrapped input and
//     computes the wrapped cells' values itself (translation invariance).
//   * BF16/F16 storage: values are widened to FP32, summed in FP32 and rounded
//     to nearest-even storage precision after every level, in LDS as in HBM.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace so2dr {

// Workgroup order.  Consecutive workgroups are dealt round-robin to the 8
// XCDs, each with its own L2; remapping gives each XCD a contiguous run of
// tiles, so neighbouring tiles' shared halo columns are fetched through the
// same L2.  The grid is padded to a multiple of 8 (xcd_grid) so that the
// permutation covers every tile; xcd_tile returns -1 for padding
// workgroups, which exit at once.
constexpr int kXcds = 8;
__host__ __device__ constexpr int64_t xcd_grid(int64_t nwg) { return (nwg + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ int xcd_tile(int wg, int nwg) {
  const int per = (nwg + kXcds - 1) / kXcds;
  const int t = (wg % kXcds) * per + wg / kXcds;
  return t < nwg ? t : -1;
}

constexpr int kMaxPts = 81;  // 2D box of radius 4

template <typename A>
struct Weights {
  A w[kMaxPts];
};

// Arguments of one launch.  Plane indices are global along the cut axis.
template <typename A>
struct TbArgs {
  const void *in;
  void *out;
  int64_t buf_z0;          // global plane stored at index 0 of in
  int64_t out_z0;          // global plane stored at index 0 of out
  int64_t plane;           // elements per plane (nx * ny)
  int nx, ny;              // in-plane extents (ny == 1 for a 2D grid)
  int per_x, per_y;        // periodic flags of the in-plane axes
  int64_t n_axis;          // length of the cut axis
  int64_t in_lo, in_hi;    // valid planes of the input level
  int64_t out_lo, out_hi;  // planes to produce at the output level
  int64_t zseg;            // output planes per workgroup segment
  int ntx, nty, nseg;      // tiles along x, y and segments along the cut axis
  Weights<A> w;
};

// ---------------------------------------------------------------- storage
template <typename T> struct Store;
template <> struct Store<float> {
  using A = float;
  static __device__ __forceinline__ float load(const float *p) { return *p; }
  static __device__ __forceinline__ void store(float *p, float v) { *p = v; }
  static __device__ __forceinline__ float round(float v) { return v; }
};
template <> struct Store<double> {
  using A = double;
  static __device__ __forceinline__ double load(const double *p) { return *p; }
  static __device__ __forceinline__ void store(double *p, double v) { *p = v; }
  static __device__ __forceinline__ double round(double v) { return v; }
};
template <> struct Store<__hip_bfloat16> {
  using A = float;
  static __device__ __forceinline__ float load(const __hip_bfloat16 *p) { return __bfloat162float(*p); }
  static __device__ __forceinline__ void store(__hip_bfloat16 *p, float v) { *p = __float2bfloat16(v); }
  static __device__ __forceinline__ float round(float v) { return __bfloat162float(__float2bfloat16(v)); }
};
// FP32 -> FP16 happens on a value pinned in a register first: otherwise the
// compiler may fuse the last FMA of a sum with the conversion into one
// mixed-precision instruction that rounds the exact value once, instead of
// the documented FP32 rounding followed by FP16 rounding -- and may do so in
// some kernels but not others, which would break schedule independence.
__device__ __forceinline__ float pin_f32(float v) {
  asm volatile("" : "+v"(v));
  return v;
}
template <> struct Store<__half> {
  using A = float;
  static __device__ __forceinline__ float load(const __half *p) { return __half2float(*p); }
  static __device__ __forceinline__ void store(__half *p, float v) { *p = __float2half(pin_f32(v)); }
  static __device__ __forceinline__ float round(float v) { return __half2float(__float2half(pin_f32(v))); }
};

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------- stencil
// Point set of a star or box stencil and the index of each (dz, dy, dx)
// offset in the lexicographic weight array (-1 when not a stencil point).
template <int NDIM, bool BOX, int R>
struct Stencil {
  static constexpr int RY = NDIM == 3 ? R : 0;  // in-plane y reach
  static constexpr int W = 2 * R + 1, WY = 2 * RY + 1;
  static constexpr bool in_set(int dz, int dy, int dx) {
    if (dz < -R || dz > R || dy < -RY || dy > RY || dx < -R || dx > R) return false;
    if (BOX) return true;
    return ((dz != 0) + (dy != 0) + (dx != 0)) <= 1;
  }
  struct Table {
    int idx[W][WY][W];
    int n;
  };
  static constexpr Table make() {
    Table t{};
    int k = 0;
    for (int a = -R; a <= R; ++a)
      for (int b = -RY; b <= RY; ++b)
        for (int c = -R; c <= R; ++c) t.idx[a + R][b + RY][c + R] = in_set(a, b, c) ? k++ : -1;
    t.n = k;
    return t;
  }
  static constexpr Table table = make();
  static constexpr int npts() { return table.n; }
  // whether any plane uses in-plane offset (dy, dx)
  static constexpr bool used_xy(int dy, int dx) {
    for (int a = -R; a <= R; ++a)
      if (in_set(a, dy, dx)) return true;
    return false;
  }
};

// Tile shape per (dimension, radius, fused depth).
template <int NDIM, int R, int KL>
struct Tile {
  static constexpr int NT = 256;
  static constexpr int TX = NDIM == 2 ? (R >= 3 ? 512 : 1024) : 64;
  static constexpr int TY = NDIM == 2 ? 1 : (KL * R <= 2 ? 16 : 32);
  static constexpr int RY = NDIM == 3 ? R : 0;
  static constexpr int NC = TX * TY / NT;  // cells per lane
  static constexpr int LX = TX + 2 * R;    // LDS row, padded by R each side
  static constexpr int LY = TY + 2 * RY;
  static constexpr int LPLANE = LX * LY;
  static constexpr int OX = TX - 2 * KL * R;  // output columns per tile
  static constexpr int OY = NDIM == 2 ? 1 : TY - 2 * KL * RY;
  static_assert(OX > 0 && OY > 0, "tile too small for this depth");
};

// RAS (round at store): levels below the last keep FP32 sums; only the value
// a launch stores is rounded to the storage type.
template <typename T, int NDIM, bool BOX, int R, int KL, bool RAS = false>
__global__ __launch_bounds__(256) void tb_kernel(const TbArgs<typename Store<T>::A> a) {
  using A = typename Store<T>::A;
  using S = Stencil<NDIM, BOX, R>;
  using G = Tile<NDIM, R, KL>;
  constexpr int RY = G::RY, TX = G::TX, NC = G::NC, LX = G::LX, W = 2 * R + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  A *lds = reinterpret_cast<A *>(smem_raw);  // [KL][2][LPLANE]

  const T *__restrict__ in = static_cast<const T *>(a.in);
  T *__restrict__ out = static_cast<T *>(a.out);

  // workgroup -> (tile x, tile y, segment)
  int wg = xcd_tile(blockIdx.x, a.ntx * a.nty * a.nseg);
  if (wg < 0) return;
  const int tx_i = wg % a.ntx;
  wg /= a.ntx;
  const int ty_i = wg % a.nty;
  const int seg = wg / a.nty;
  const int64_t zo0 = a.out_lo + (int64_t)seg * a.zseg;
  if (zo0 >= a.out_hi) return;  // uniform for the whole workgroup
  const int64_t zo1 = (zo0 + a.zseg < a.out_hi) ? zo0 + a.zseg : a.out_hi;
  const int64_t P0 = zo0 - (int64_t)KL * R;  // first input plane
  const int gx0 = tx_i * G::OX - KL * R;     // extended coordinate of tile column 0
  const int gy0 = ty_i * G::OY - KL * RY;

  // per-cell constants
  int lidx[NC];       // LDS index of the cell (padded layout)
  int goff[NC];       // in-plane element offset of its (wrapped) source cell
  bool ghost[NC];     // outside the grid on a Dirichlet axis: zero at all levels
  bool outc[NC];      // written at the output level
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int L = threadIdx.x + G::NT * c;
    const int x = L % TX, y = L / TX;
    lidx[c] = (y + RY) * LX + (x + R);
    int gx = gx0 + x, gy = gy0 + y;
    bool gh = false;
    if (gx < 0 || gx >= a.nx) {
      if (a.per_x) gx = ((gx % a.nx) + a.nx) % a.nx; else gh = true;
    }
    if (gy < 0 || gy >= a.ny) {
      if (a.per_y) gy = ((gy % a.ny) + a.ny) % a.ny; else gh = true;
    }
    ghost[c] = gh;
    goff[c] = gh ? 0 : gy * a.nx + gx;
    const int ox = gx0 + x, oy = gy0 + y;
    outc[c] = !gh && x >= KL * R && x < TX - KL * R && y >= KL * RY && y < G::TY - KL * RY &&
              ox < a.nx && oy < a.ny;
  }

  A acc[KL][NC][W];   // partial sums; acc[l][c][k] belongs to output p + R - k
  A done[KL][NC];     // newest completed plane of levels 1..KL-1 (index 0 unused)
  A nxt[NC];          // prefetched input plane
#pragma unroll
  for (int l = 0; l < KL; ++l)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      done[l][c] = A(0);
#pragma unroll
      for (int k = 0; k < W; ++k) acc[l][c][k] = A(0);
    }

  const int64_t span = zo1 - zo0;
  const int64_t n_load = span + 2 * KL * R;
  const int64_t n_steps = span + 2 * KL * R + KL - 1;

  auto load_plane = [&](int64_t p, A *dst) {
    const bool ok = p >= a.in_lo && p < a.in_hi && p >= 0 && p < a.n_axis;
    const T *base = in + (p - a.buf_z0) * a.plane;
#pragma unroll
    for (int c = 0; c < NC; ++c) dst[c] = (ok && !ghost[c]) ? Store<T>::load(base + goff[c]) : A(0);
  };

  load_plane(P0, nxt);

  for (int64_t m = 0; m < n_steps; ++m) {
    const int b = (int)(m & 1);
    // ---- publish: level 0 = the input plane P0 + m; level l = done[l]
    if (m < n_load) {
      A *dst = lds + (0 * 2 + b) * G::LPLANE;
#pragma unroll
      for (int c = 0; c < NC; ++c) dst[lidx[c]] = nxt[c];
      if (m + 1 < n_load) load_plane(P0 + m + 1, nxt);
    }
#pragma unroll
    for (int l = 1; l < KL; ++l) {
      A *dst = lds + (l * 2 + b) * G::LPLANE;
#pragma unroll
      for (int c = 0; c < NC; ++c) dst[lidx[c]] = done[l][c];
    }
    __syncthreads();
    // ---- consume: level l takes the plane level l-1 published this step
#pragma unroll
    for (int l = 1; l <= KL; ++l) {
      // plane of level l-1 in LDS this step, relative to P0
      const int64_t e = m - (int64_t)(l - 1) * (R + 1);
      const bool useful = e >= (int64_t)(l - 1) * R && e < span + (int64_t)(2 * KL - l + 1) * R;
      if (!useful) continue;  // uniform branch
      const A *src = lds + ((l - 1) * 2 + b) * G::LPLANE;
      const int64_t q = P0 + e - R;  // plane completed by this consumption
      const bool zghost = q < 0 || q >= a.n_axis;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        A v[2 * RY + 1][W];
#pragma unroll
        for (int dy = -RY; dy <= RY; ++dy)
#pragma unroll
          for (int dx = -R; dx <= R; ++dx) {
            v[dy + RY][dx + R] = S::used_xy(dy, dx) ? src[lidx[c] + dy * LX + dx] : A(0);
          }
        // output p - dz receives this plane's dz terms; k = R + dz
#pragma unroll
        for (int dz = -R; dz <= R; ++dz) {
          A s = acc[l - 1][c][R + dz];
#pragma unroll
          for (int dy = -RY; dy <= RY; ++dy)
#pragma unroll
            for (int dx = -R; dx <= R; ++dx) {
              const int wi = S::table.idx[dz + R][dy + RY][dx + R];
              if (wi >= 0) s = fma_(a.w.w[wi], v[dy + RY][dx + R], s);
            }
          acc[l - 1][c][R + dz] = s;
        }
        A res = RAS && l < KL ? acc[l - 1][c][2 * R] : Store<T>::round(acc[l - 1][c][2 * R]);
        if (zghost || ghost[c]) res = A(0);
        // rotate: output p + R - k moves to slot k + 1
#pragma unroll
        for (int k = 2 * R; k > 0; --k) acc[l - 1][c][k] = acc[l - 1][c][k - 1];
        acc[l - 1][c][0] = A(0);
        if (l < KL) {
          done[l][c] = res;
        } else if (outc[c] && q >= zo0 && q < zo1) {
          Store<T>::store(out + (q - a.out_z0) * a.plane + goff[c], res);
        }
      }
    }
  }
}

template <typename T, int NDIM, bool BOX, int R, int KL>
constexpr size_t tb_lds_bytes() {
  using G = Tile<NDIM, R, KL>;
  return sizeof(typename Store<T>::A) * (size_t)KL * 2 * G::LPLANE;
}

}  // namespace so2dr
