// march_kernel.hpp -- fused-step kernel for 3D star and box stencils with the
// march along the cut axis unrolled by the stencil width.
//
// Same contract and the same per-cell arithmetic as tb_kernel and
// col3d_kernel (each output's FMA chain starts from +0 and runs over the
// points in lexicographic (dz, dy, dx) order, per-level rounding to storage),
// so all three give identical bits.  What this one changes is the cost per
// march step, which decides whether a fused launch keeps up with HBM:
//   * the 2R+1 partial sums of a cell live in a ring indexed by output plane
//     modulo 2R+1; the march loop is unrolled by 2R+1 steps, so every ring
//     index is a compile-time constant and nothing is moved between
//     registers.  An output's first term starts its sum from +0 directly;
//   * prefetched input planes sit in a ring of RS slots, RS the smallest
//     multiple of 2R+1 above PF (plane p in slot p mod RS; the march is
//     unrolled by RS), loaded PF steps ahead without conditions: the plane
//     index is clamped into the buffer's valid planes and every lane reads an
//     in-grid address (ghost columns and rows read a clamped or wrapped one),
//     so a load's destination is the ring register itself.  Ghost values are
//     set to zero when a plane is consumed, in a second copy of the march
//     that only workgroups touching a Dirichlet boundary run;
//   * all march arithmetic on plane indices is 32-bit and uniform, and each
//     row is addressed as a per-plane base plus one 32-bit byte offset;
//   * a lane owns VX consecutive x cells (VX = 4: 1 KiB FP32 rows, 16-byte
//     accesses), a wave M rows, a workgroup NW waves stacked in y; x
//     neighbours across lanes come from whole-wave DPP shifts, y neighbours
//     across waves from LDS (HB = 2: double-buffered, one barrier per step;
//     HB = 1: one buffer and a second barrier before it is overwritten).
//
// Requirements checked by the launcher: nx % VX == 0, a plane's bytes below
// 2^32 and plane indices below 2^30.  Planes outside [in_lo, in_hi) but
// inside the grid hold stale values here rather than zeros: only outputs
// outside the compute area, which are never stored, depend on them.
#pragma once
#include <utility>

#include "star_kernel.hpp"

namespace so2dr {

template <int V>
using IC = std::integral_constant<int, V>;

template <typename F, int... I>
__device__ __forceinline__ void unroll_seq(F &&f, std::integer_sequence<int, I...>) {
  (f(IC<I>{}), ...);
}

constexpr int pmod(int a, int m) { return ((a % m) + m) % m; }

template <typename T, bool BOX, int R, int KL, int NW, int M, int VX, int HB, int PF, bool RAS, bool GH, int HA>
__device__ __forceinline__ void march3d_tile(const TbArgs<typename Store<T>::A> &a,
                                             typename Store<T>::A (*halo)[HB][NW][2 * R][64 * VX],
                                             int lane, int wave, int tx_i, int ty_i, int zo0, int zo1);

// WPE: waves per SIMD the register allocation must allow (caps VGPRs at
// 512 / WPE).  RAS (round at store): levels below the last keep FP32 sums;
// only the value a launch stores is rounded to the storage type.
// HA: x-halo alignment in cells (StarTile).
template <typename T, bool BOX, int R, int KL, int NW, int M, int VX, int HB, int PF, int WPE = 1, bool RAS = false,
          int HA = VX>
__global__ __launch_bounds__(NW * 64, WPE) void march3d_kernel(const TbArgs<typename Store<T>::A> a) {
  using A = typename Store<T>::A;
  using G = StarTile<R, KL, NW, M, VX, HA>;
  __shared__ A halo[KL][HB][NW][2 * R][64 * VX];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  int wg = xcd_tile(blockIdx.x, a.ntx * a.nty * a.nseg);
  if (wg < 0) return;
  const int tx_i = wg % a.ntx;
  wg /= a.ntx;
  const int ty_i = wg % a.nty;
  const int seg = wg / a.nty;
  const int zo0 = (int)a.out_lo + seg * (int)a.zseg;
  if (zo0 >= (int)a.out_hi) return;
  const int zo1 = min(zo0 + (int)a.zseg, (int)a.out_hi);
  // ghost cells anywhere in this workgroup's work: Dirichlet columns or rows
  // in the tile, or planes outside the grid along the cut axis (uniform)
  const int x_lo = tx_i * G::OX - G::HX, y_lo = ty_i * G::OY - G::HY;
  // (the march consumes planes [P0, P0 + n_load) and produces level planes
  // from P0 - R on; one more R of margin on each side)
  const int P0 = zo0 - KL * R, n_load = zo1 - zo0 + 2 * KL * R;
  const bool ghosts = (!a.per_x && (x_lo < 0 || x_lo + G::TX > a.nx)) ||
                      (!a.per_y && (y_lo < 0 || y_lo + G::TY > a.ny)) || P0 - 2 * R < 0 ||
                      P0 + n_load + R > (int)a.n_axis;
  if (ghosts)
    march3d_tile<T, BOX, R, KL, NW, M, VX, HB, PF, RAS, true, HA>(a, halo, lane, wave, tx_i, ty_i, zo0, zo1);
  else
    march3d_tile<T, BOX, R, KL, NW, M, VX, HB, PF, RAS, false, HA>(a, halo, lane, wave, tx_i, ty_i, zo0, zo1);
}

template <typename T, bool BOX, int R, int KL, int NW, int M, int VX, int HB, int PF, bool RAS, bool GH, int HA>
__device__ __forceinline__ void march3d_tile(const TbArgs<typename Store<T>::A> &a,
                                             typename Store<T>::A (*halo)[HB][NW][2 * R][64 * VX],
                                             int lane, int wave, int tx_i, int ty_i, int zo0, int zo1) {
  using A = typename Store<T>::A;
  using S = Stencil<3, BOX, R>;
  using G = StarTile<R, KL, NW, M, VX, HA>;
  constexpr int W = 2 * R + 1;
  constexpr int RS = W * (PF / W + 1);  // prefetch ring: a multiple of W above PF
  static_assert(PF >= 1 && PF < RS, "prefetch distance must leave the consumed slot alone");
  const int P0 = zo0 - KL * R;
  const int n_axis = (int)a.n_axis;
  const int p_lo = max((int)a.in_lo, 0), p_hi = min((int)a.in_hi, n_axis) - 1;  // loadable planes
  const int x_lo = tx_i * G::OX - G::HX, y_lo = ty_i * G::OY - G::HY;

  const T *__restrict__ in = static_cast<const T *>(a.in);
  T *__restrict__ out = static_cast<T *>(a.out);
  const int cx0 = lane * VX;
  const int gx0 = x_lo + cx0;  // VX-aligned: x_lo and cx0 are multiples of VX
  int lx = gx0;
  bool keep_x = true;
  if (gx0 < 0 || gx0 >= a.nx) {
    if (a.per_x) lx = ((gx0 % a.nx) + a.nx) % a.nx; else { lx = 0; keep_x = false; }
  }
  const bool out_lane = cx0 >= G::HX && cx0 < G::TX - G::HX && gx0 < a.nx;
  uint32_t boff[M];
  bool keep[M], st[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int t = wave * M + m;
    const int gy = y_lo + t;
    int ly = gy;
    bool keep_y = true;
    if (gy < 0 || gy >= a.ny) {
      if (a.per_y) ly = ((gy % a.ny) + a.ny) % a.ny; else { ly = 0; keep_y = false; }
    }
    boff[m] = (uint32_t)(ly * a.nx + lx) * (uint32_t)sizeof(T);
    keep[m] = keep_x && keep_y;
    st[m] = out_lane && t >= G::HY && t < G::TY - G::HY && gy < a.ny;
  }

  A acc[KL][M][VX][W];  // acc[l][m][j][o mod W]: partial sum of output plane o
  A done[KL][M][VX];    // newest completed plane of levels 1..KL-1
  A ring[RS][M][VX];    // input plane P0 + p in slot p mod RS
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

  const int span = zo1 - zo0;
  const int n_load = span + 2 * KL * R;
  // steps past the last useful one are no-ops for every level, so the count
  // is rounded up to whole unrolled groups
  const int n_steps = (n_load + KL - 1 + RS - 1) / RS * RS;

  auto load_plane = [&](int p, A (*dst)[VX]) {
    const int pc = min(max(p, p_lo), p_hi);
    const char *base = reinterpret_cast<const char *>(in + (int64_t)(pc - (int)a.buf_z0) * a.plane);
#pragma unroll
    for (int m = 0; m < M; ++m) VecIO<T, VX>::load(reinterpret_cast<const T *>(base + boff[m]), dst[m]);
  };
#pragma unroll
  for (int k = 0; k < PF; ++k) load_plane(P0 + k, ring[k]);

  const int wu = wave > 0 ? wave - 1 : 0;  // clamped: rows beyond the tile are never valid
  const int wd = wave < NW - 1 ? wave + 1 : NW - 1;

  // one march step; s = PH (mod RS), so also s = PH (mod W)
  auto step = [&](auto ph_c, int s) {
    constexpr int PH = decltype(ph_c)::value;
    const int b = HB == 2 ? (s & 1) : 0;
    if (HB == 1) __syncthreads();  // the previous step's halo reads are done
    load_plane(P0 + s + PF, ring[(PH + PF) % RS]);
    if constexpr (GH) {  // ghosts of the plane consumed now
      const bool zg = P0 + s < 0 || P0 + s >= n_axis;
#pragma unroll
      for (int m = 0; m < M; ++m)
#pragma unroll
        for (int j = 0; j < VX; ++j) ring[PH][m][j] = keep[m] && !zg ? ring[PH][m][j] : A(0);
    }
    // publish the boundary rows of every level's newest plane
#pragma unroll
    for (int l = 0; l < KL; ++l)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < VX; ++j) {
          halo[l][b][wave][r][cx0 + j] = l == 0 ? ring[PH][r][j] : done[l][r][j];
          halo[l][b][wave][R + r][cx0 + j] = l == 0 ? ring[PH][M - R + r][j] : done[l][M - R + r][j];
        }
    __syncthreads();
    // deepest level first: each consumes its predecessor's plane of the
    // previous step before that register is overwritten
    unroll_seq(
        [&](auto li) {
          constexpr int l = KL - decltype(li)::value;  // KL .. 1
          const int e = s - (l - 1) * (R + 1);           // consumed plane, relative to P0
          if (!(e >= (l - 1) * R && e < span + (2 * KL - l + 1) * R)) return;
          constexpr int EP = pmod(PH - (l - 1) * (R + 1), W);  // e mod W
          const int q = P0 + e - R;                              // plane completed now
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
            for (int j = 0; j < VX; ++j) col[R + m][j] = l == 1 ? ring[PH][m][j] : done[l - 1][m][j];
          A row[M + 2 * R][VX + 2 * R];
#pragma unroll
          for (int i = 0; i < M + 2 * R; ++i) {
#pragma unroll
            for (int j = 0; j < VX; ++j) row[i][R + j] = col[i][j];
#pragma unroll
            for (int k = 1; k <= R; ++k) {
              const int sh = (k + VX - 1) / VX;
              const A lv = col[i][VX * sh - k], rv = col[i][k - 1 - VX * (sh - 1)];
              row[i][R - k] = sh == 1 ? dpp_f<kDppWaveShr1>(lv) : dpp_f<kDppWaveShr1>(dpp_f<kDppWaveShr1>(lv));
              row[i][R + VX - 1 + k] =
                  sh == 1 ? dpp_f<kDppWaveShl1>(rv) : dpp_f<kDppWaveShl1>(dpp_f<kDppWaveShl1>(rv));
            }
          }
          A res[M][VX];
#pragma unroll
          for (int m = 0; m < M; ++m)
#pragma unroll
            for (int j = 0; j < VX; ++j) {
#pragma unroll
              for (int dz = -R; dz <= R; ++dz) {
                const int slot = pmod(EP - dz, W);  // output e - dz
                A sum = dz == -R ? A(0) : acc[l - 1][m][j][slot];
#pragma unroll
                for (int dy = -R; dy <= R; ++dy)
#pragma unroll
                  for (int dx = -R; dx <= R; ++dx) {
                    const int wi = S::table.idx[dz + R][dy + R][dx + R];
                    if (wi >= 0) sum = fma_(a.w.w[wi], row[R + m + dy][R + j + dx], sum);
                  }
                acc[l - 1][m][j][slot] = sum;
              }
              const A v = acc[l - 1][m][j][pmod(EP - R, W)];
              res[m][j] = RAS && l < KL ? v : Store<T>::round(v);
            }
          if constexpr (GH) {
            const bool zg = q < 0 || q >= n_axis;
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
              for (int j = 0; j < VX; ++j) res[m][j] = keep[m] && !zg ? res[m][j] : A(0);
          }
          if constexpr (l < KL) {
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
              for (int j = 0; j < VX; ++j) done[l][m][j] = res[m][j];
          } else {
            if (q >= zo0 && q < zo1) {
              char *dst = reinterpret_cast<char *>(out + (int64_t)(q - (int)a.out_z0) * a.plane);
#pragma unroll
              for (int m = 0; m < M; ++m)
                if (st[m]) VecIO<T, VX>::store(reinterpret_cast<T *>(dst + boff[m]), res[m]);
            }
          }
        },
        std::make_integer_sequence<int, KL>{});
  };

  for (int s = 0; s < n_steps; s += RS)
    unroll_seq([&](auto ph) { step(ph, s + decltype(ph)::value); }, std::make_integer_sequence<int, RS>{});
}

}  // namespace so2dr
