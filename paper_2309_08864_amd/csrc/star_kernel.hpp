// star_kernel.hpp -- register-column fused-step kernel for 3D star and box
// stencils.
//
// Same contract and the same per-cell arithmetic as tb_kernel (each output's
// FMA chain in lexicographic (dz, dy, dx) order, partial sums advanced as
// planes arrive, per-level rounding to storage), so the two give identical
// bits; this one is organised for MI355X's memory system:
//   * a lane owns VX consecutive x cells, so a wave row is 64 VX cells (1 KiB
//     of FP32 for VX = 4) read and written with vector accesses -- wide
//     contiguous rows are what HBM streams well; the tile's x halo is rounded
//     up to whole lanes so every vector access stays aligned;
//   * a wave owns M consecutive y rows; a lane keeps its VX x M cells of every
//     level in registers, so y-neighbours inside the wave never leave it;
//   * x-neighbours across lanes come from whole-wave DPP lane shifts
//     (wave_shr / wave_shl): no LDS traffic in x;
//   * only the R rows at each wave boundary go through LDS (double-buffered
//     with one barrier per march step, or single-buffered with two);
//   * input planes are prefetched two march steps ahead into registers.
#pragma once
#include <type_traits>

#include "tb_kernel.hpp"

namespace so2dr {

// DPP control codes of the whole-wave shifts (GFX9 DPP): lane i receives lane
// i-1 (shift right) or lane i+1 (shift left); the lane without a source gets 0.
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// VX consecutive stored elements <-> VX values of the accumulation type, in
// one vector access (the caller guarantees alignment)
template <typename T, int VX> struct VecIO;
template <int VX> struct VecIO<float, VX> {
  using V = typename std::conditional<VX == 4, float4, float2>::type;
  static __device__ __forceinline__ void load(const float *p, float *v) {
    const V q = *reinterpret_cast<const V *>(p);
    __builtin_memcpy(v, &q, sizeof(V));
  }
  static __device__ __forceinline__ void store(float *p, const float *v) {
    V q;
    __builtin_memcpy(&q, v, sizeof(V));
    *reinterpret_cast<V *>(p) = q;
  }
};
template <int VX> struct VecIO<double, VX> {
  static __device__ __forceinline__ void load(const double *p, double *v) {
#pragma unroll
    for (int i = 0; i < VX; i += 2) {
      const double2 q = reinterpret_cast<const double2 *>(p)[i / 2];
      v[i] = q.x;
      v[i + 1] = q.y;
    }
  }
  static __device__ __forceinline__ void store(double *p, const double *v) {
#pragma unroll
    for (int i = 0; i < VX; i += 2) reinterpret_cast<double2 *>(p)[i / 2] = make_double2(v[i], v[i + 1]);
  }
};
template <typename H16, int VX> struct VecIOHalf {
  using V = typename std::conditional<VX == 4, uint2, unsigned>::type;
  static __device__ __forceinline__ void load(const H16 *p, float *v) {
    const V q = *reinterpret_cast<const V *>(p);
    unsigned short bits[VX];
    __builtin_memcpy(bits, &q, sizeof(V));
#pragma unroll
    for (int i = 0; i < VX; ++i) {
      H16 h;
      __builtin_memcpy(&h, &bits[i], 2);
      v[i] = Store<H16>::load(&h);
    }
  }
  static __device__ __forceinline__ void store(H16 *p, const float *v) {
    unsigned short bits[VX];
#pragma unroll
    for (int i = 0; i < VX; ++i) {
      H16 h;
      Store<H16>::store(&h, v[i]);
      __builtin_memcpy(&bits[i], &h, 2);
    }
    V q;
    __builtin_memcpy(&q, bits, sizeof(V));
    *reinterpret_cast<V *>(p) = q;
  }
};
template <int VX> struct VecIO<__hip_bfloat16, VX> : VecIOHalf<__hip_bfloat16, VX> {};
template <int VX> struct VecIO<__half, VX> : VecIOHalf<__half, VX> {};
// one cell per lane: plain scalar accesses
template <> struct VecIO<float, 1> {
  static __device__ __forceinline__ void load(const float *p, float *v) { v[0] = *p; }
  static __device__ __forceinline__ void store(float *p, const float *v) { *p = v[0]; }
};
template <> struct VecIO<double, 1> {
  static __device__ __forceinline__ void load(const double *p, double *v) { v[0] = *p; }
  static __device__ __forceinline__ void store(double *p, const double *v) { *p = v[0]; }
};
template <> struct VecIO<__hip_bfloat16, 1> {
  static __device__ __forceinline__ void load(const __hip_bfloat16 *p, float *v) { v[0] = Store<__hip_bfloat16>::load(p); }
  static __device__ __forceinline__ void store(__hip_bfloat16 *p, const float *v) { Store<__hip_bfloat16>::store(p, v[0]); }
};
template <> struct VecIO<__half, 1> {
  static __device__ __forceinline__ void load(const __half *p, float *v) { v[0] = Store<__half>::load(p); }
  static __device__ __forceinline__ void store(__half *p, const float *v) { Store<__half>::store(p, v[0]); }
};

// HA: the x halo is rounded up to a multiple of HA cells (whole lanes at
// least); with 64-cell-multiple rows and a 64-byte halo the output rows of
// every tile start and end on 128-byte lines.
template <int R, int KL, int NW, int M, int VX_, int HA = VX_>
struct StarTile {
  static constexpr int VX = VX_;                        // x cells per lane
  static constexpr int TX = 64 * VX, TY = NW * M;
  static constexpr int HX = (KL * R + HA - 1) / HA * HA;  // x halo
  static_assert(HA % VX == 0, "the x halo must be whole lanes");
  static constexpr int HY = KL * R;
  static constexpr int OX = TX - 2 * HX, OY = TY - 2 * HY;
  static_assert(M >= R && R <= 2 * VX && OX > 0 && OY > 0, "tile too small for this depth");
};

template <typename T, bool BOX, int R, int KL, int NW, int M, int VX_, int HB, bool RAS = false>
__global__ __launch_bounds__(NW * 64) void col3d_kernel(const TbArgs<typename Store<T>::A> a) {
  using A = typename Store<T>::A;
  using S = Stencil<3, BOX, R>;
  using G = StarTile<R, KL, NW, M, VX_>;
  constexpr int W = 2 * R + 1, VX = G::VX;
  // wave boundary rows (top R then bottom R) of every level; HB = 2 buffers
  // alternate by step (one barrier per step), HB = 1 needs a second barrier
  __shared__ A halo[KL][HB][NW][2 * R][64 * VX];

  const T *__restrict__ in = static_cast<const T *>(a.in);
  T *__restrict__ out = static_cast<T *>(a.out);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  int wg = xcd_tile(blockIdx.x, a.ntx * a.nty * a.nseg);
  if (wg < 0) return;
  const int tx_i = wg % a.ntx;
  wg /= a.ntx;
  const int ty_i = wg % a.nty;
  const int seg = wg / a.nty;
  const int64_t zo0 = a.out_lo + (int64_t)seg * a.zseg;
  if (zo0 >= a.out_hi) return;
  const int64_t zo1 = (zo0 + a.zseg < a.out_hi) ? zo0 + a.zseg : a.out_hi;
  const int64_t P0 = zo0 - (int64_t)KL * R;

  // this lane's 4 columns
  const int cx0 = lane * VX;                      // tile column of cell 0
  const int gx0 = tx_i * G::OX - G::HX + cx0;     // grid column of cell 0 (unreduced)
  int gxc[VX];
  bool ghx[VX], outx[VX];
  bool inside_all = true;
#pragma unroll
  for (int j = 0; j < VX; ++j) {
    int gx = gx0 + j;
    const bool in_grid = gx >= 0 && gx < a.nx;
    inside_all &= in_grid;
    ghx[j] = !in_grid && !a.per_x;
    if (!in_grid && a.per_x) gx = ((gx % a.nx) + a.nx) % a.nx;
    gxc[j] = ghx[j] ? 0 : gx;
    outx[j] = cx0 + j >= G::HX && cx0 + j < G::TX - G::HX && gx0 + j < a.nx;
  }
  // vector accesses need the VX cells inside the grid and VX-aligned rows
  const bool vec = inside_all && (a.nx % VX) == 0;
  const bool out_vec = vec && outx[0] && outx[VX - 1];
  int rowoff[M];
  bool ghy[M], outy[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int t = wave * M + m;
    const int gy_raw = ty_i * G::OY - G::HY + t;
    int gy = gy_raw;
    ghy[m] = false;
    if (gy < 0 || gy >= a.ny) {
      if (a.per_y) gy = ((gy % a.ny) + a.ny) % a.ny; else ghy[m] = true;
    }
    rowoff[m] = ghy[m] ? 0 : gy * a.nx;
    outy[m] = !ghy[m] && t >= G::HY && t < G::TY - G::HY && gy_raw < a.ny;
  }

  A acc[KL][M][VX][W];
  A done[KL][M][VX];  // newest completed plane of levels 1..KL-1
  A cur[M][VX], pf0[M][VX], pf1[M][VX];
#pragma unroll
  for (int l = 0; l < KL; ++l)
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int j = 0; j < VX; ++j) {
        done[l][m][j] = A(0);
#pragma unroll
        for (int k = 0; k < W; ++k) acc[l][m][j][k] = A(0);
      }

  const int64_t span = zo1 - zo0;
  const int64_t n_load = span + 2 * KL * R;
  const int64_t n_steps = n_load + KL - 1;

  auto load_plane = [&](int64_t p, A (*dst)[VX]) {
    const bool ok = p >= a.in_lo && p < a.in_hi && p >= 0 && p < a.n_axis;
    const T *base = in + (p - a.buf_z0) * a.plane;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (ok && !ghy[m] && vec) {
        VecIO<T, VX>::load(base + rowoff[m] + gx0, dst[m]);
      } else {
#pragma unroll
        for (int j = 0; j < VX; ++j)
          dst[m][j] = (ok && !ghy[m] && !ghx[j]) ? Store<T>::load(base + rowoff[m] + gxc[j]) : A(0);
      }
    }
  };
  load_plane(P0, pf0);
  if (n_load > 1) load_plane(P0 + 1, pf1);

  const int wu = wave > 0 ? wave - 1 : 0;  // neighbours (clamped: rows outside the tile are garbage)
  const int wd = wave < NW - 1 ? wave + 1 : NW - 1;

  for (int64_t step = 0; step < n_steps; ++step) {
    const int b = HB == 2 ? (int)(step & 1) : 0;
    if (HB == 1 && step > 0) __syncthreads();  // last step's halo reads are done
    if (step < n_load) {
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int j = 0; j < VX; ++j) {
          cur[m][j] = pf0[m][j];
          pf0[m][j] = pf1[m][j];
        }
      if (step + 2 < n_load) load_plane(P0 + step + 2, pf1);
    }
    // publish the boundary rows of every level's newest plane
#pragma unroll
    for (int l = 0; l < KL; ++l)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < VX; ++j) {
          halo[l][b][wave][r][cx0 + j] = l == 0 ? cur[r][j] : done[l][r][j];
          halo[l][b][wave][R + r][cx0 + j] = l == 0 ? cur[M - R + r][j] : done[l][M - R + r][j];
        }
    __syncthreads();
    // deepest level first, so each consumes its predecessor's plane from the
    // previous step before that register is overwritten
#pragma unroll
    for (int l = KL; l >= 1; --l) {
      const int64_t e = step - (int64_t)(l - 1) * (R + 1);
      const bool useful = e >= (int64_t)(l - 1) * R && e < span + (int64_t)(2 * KL - l + 1) * R;
      if (!useful) continue;  // uniform branch
      const int64_t q = P0 + e - R;
      const bool zghost = q < 0 || q >= a.n_axis;
      // the consumed plane on this lane's columns, R rows above and below
      A col[M + 2 * R][VX];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < VX; ++j) {
          col[r][j] = halo[l - 1][b][wu][R + r][cx0 + j];
          col[M + R + r][j] = halo[l - 1][b][wd][r][cx0 + j];
        }
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int j = 0; j < VX; ++j) col[R + m][j] = l == 1 ? cur[m][j] : done[l - 1][m][j];
      // every row of the consumed plane, extended by R cells from each
      // neighbouring lane (unused extensions are dead code for stars)
      A row[M + 2 * R][VX + 2 * R];
#pragma unroll
      for (int i = 0; i < M + 2 * R; ++i) {
#pragma unroll
        for (int j = 0; j < VX; ++j) row[i][R + j] = col[i][j];
        // the cell k to the left of this lane's first cell sits in lane
        // -ceil(k/VX) at element VX*ceil(k/VX) - k; symmetrically on the right
#pragma unroll
        for (int k = 1; k <= R; ++k) {
          const int sh = (k + VX - 1) / VX;
          const A lv = col[i][VX * sh - k], rv = col[i][k - 1 - VX * (sh - 1)];
          row[i][R - k] = sh == 1 ? dpp_f<kDppWaveShr1>(lv) : dpp_f<kDppWaveShr1>(dpp_f<kDppWaveShr1>(lv));
          row[i][R + VX - 1 + k] = sh == 1 ? dpp_f<kDppWaveShl1>(rv) : dpp_f<kDppWaveShl1>(dpp_f<kDppWaveShl1>(rv));
        }
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
        A res_row[VX];
#pragma unroll
        for (int j = 0; j < VX; ++j) {
          // the plane's terms for each output it feeds, lexicographic (dy, dx)
#pragma unroll
          for (int dz = -R; dz <= R; ++dz) {
            A s = acc[l - 1][m][j][R + dz];
#pragma unroll
            for (int dy = -R; dy <= R; ++dy)
#pragma unroll
              for (int dx = -R; dx <= R; ++dx) {
                const int wi = S::table.idx[dz + R][dy + R][dx + R];
                if (wi >= 0) s = fma_(a.w.w[wi], row[R + m + dy][R + j + dx], s);
              }
            acc[l - 1][m][j][R + dz] = s;
          }
          A res = RAS && l < KL ? acc[l - 1][m][j][2 * R] : Store<T>::round(acc[l - 1][m][j][2 * R]);
          if (zghost || ghy[m] || ghx[j]) res = A(0);
#pragma unroll
          for (int k = 2 * R; k > 0; --k) acc[l - 1][m][j][k] = acc[l - 1][m][j][k - 1];
          acc[l - 1][m][j][0] = A(0);
          if (l < KL) done[l][m][j] = res;
          else res_row[j] = res;
        }
        if (l == KL && outy[m] && q >= zo0 && q < zo1) {
          T *dst = out + (q - a.out_z0) * a.plane + rowoff[m];
          if (out_vec) {
            VecIO<T, VX>::store(dst + gx0, res_row);
          } else {
#pragma unroll
            for (int j = 0; j < VX; ++j)
              if (outx[j] && !ghx[j]) Store<T>::store(dst + gxc[j], res_row[j]);
          }
        }
      }
    }
  }
}

}  // namespace so2dr
