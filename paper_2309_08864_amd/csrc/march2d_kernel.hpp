// march2d_kernel.hpp -- fused-step kernel for 2D star and box stencils: one
// wave per tile, no LDS and no barriers.
//
// Same contract and the same per-cell arithmetic as tb_kernel (each output's
// FMA chain starts from +0 and runs over the points in lexicographic order of
// (cut-axis offset, x offset), per-level rounding to storage), so the two give
// identical bits.  In 2D a "plane" of the march is one row, so a wave can own
// a whole tile:
//   * a lane owns VX consecutive cells of the row; the wave's 64 VX cells
//     overlap the neighbouring tiles by KL R cells per side (rounded up to
//     whole lanes), the redundant tile-edge work of on-chip blocking;
//   * x neighbours come from whole-wave DPP shifts, so rows never leave the
//     registers and the waves of a workgroup never wait for each other;
//   * per level and cell, 2R+1 partial sums in a ring indexed by output row
//     modulo 2R+1, with the march unrolled by 2R+1 rows so that every ring
//     index is a compile-time constant (ROT = false); where that unrolled
//     body would be too large for the instruction cache (wide box stencils
//     at depth), the sums shift by one register per row instead (ROT = true)
//     and the march is unrolled only by the prefetch ring's width;
//   * input rows are prefetched PF rows ahead into a ring of the same width,
//     unconditionally: the row index is clamped into the buffer's valid rows
//     and ghost columns read a clamped or wrapped in-grid address; ghosts are
//     zeroed in a second copy of the march that only waves touching a
//     Dirichlet boundary run.
// Requirements checked by the launcher: nx % VX == 0, row bytes and row
// indices within 32 bits.  Rows outside [in_lo, in_hi) but inside the grid
// hold stale values here rather than zeros: only outputs outside the compute
// area, which are never stored, depend on them.
#pragma once
#include "march_kernel.hpp"

namespace so2dr {

template <int R, int KL, int VX>
struct RowTile {
  static constexpr int TX = 64 * VX;
  static constexpr int HX = (KL * R + VX - 1) / VX * VX;
  static constexpr int OX = TX - 2 * HX;
  static_assert(R <= 2 * VX && OX > 0, "tile too small for this depth");
};

template <typename T, bool BOX, int R, int KL, int VX, int PF, bool ROT, bool RAS, bool GH>
__device__ __forceinline__ void march2d_tile(const TbArgs<typename Store<T>::A> &a, int lane, int tx_i,
                                             int zo0, int zo1) {
  using A = typename Store<T>::A;
  using S = Stencil<2, BOX, R>;
  using G = RowTile<R, KL, VX>;
  constexpr int W = 2 * R + 1;
  static_assert(PF >= 1 && PF < W, "prefetch distance must leave the consumed slot alone");
  const int P0 = zo0 - KL * R;
  const int n_axis = (int)a.n_axis;
  const int p_lo = max((int)a.in_lo, 0), p_hi = min((int)a.in_hi, n_axis) - 1;
  const T *__restrict__ in = static_cast<const T *>(a.in);
  T *__restrict__ out = static_cast<T *>(a.out);

  const int cx0 = lane * VX;
  const int gx0 = tx_i * G::OX - G::HX + cx0;  // VX-aligned
  int lx = gx0;
  bool keep = true;
  if (gx0 < 0 || gx0 >= a.nx) {
    if (a.per_x) lx = ((gx0 % a.nx) + a.nx) % a.nx; else { lx = 0; keep = false; }
  }
  const bool st = cx0 >= G::HX && cx0 < G::TX - G::HX && gx0 < a.nx;
  const uint32_t boff = (uint32_t)lx * (uint32_t)sizeof(T);

  constexpr int NR = ROT ? PF + 1 : W;  // input ring slots: row P0 + p in slot p mod NR
  constexpr int U = NR;                 // rows per unrolled group
  A acc[KL][VX][W];  // ROT: acc[l][j][R + dz] feeds output e - dz; else slot o mod W
  A done[KL][VX];    // newest completed row of levels 1..KL-1
  A ring[NR][VX];
#pragma unroll
  for (int l = 0; l < KL; ++l)
#pragma unroll
    for (int j = 0; j < VX; ++j) {
      done[l][j] = A(0);
#pragma unroll
      for (int k = 0; k < W; ++k) acc[l][j][k] = A(0);
    }
  const int span = zo1 - zo0;
  const int n_load = span + 2 * KL * R;
  const int n_steps = (n_load + KL - 1 + U - 1) / U * U;

  auto load_row = [&](int p, A *dst) {
    const int pc = min(max(p, p_lo), p_hi);
    const char *base = reinterpret_cast<const char *>(in + (int64_t)(pc - (int)a.buf_z0) * a.plane);
    VecIO<T, VX>::load(reinterpret_cast<const T *>(base + boff), dst);
  };
#pragma unroll
  for (int k = 0; k < PF; ++k) load_row(P0 + k, ring[k]);

  auto step = [&](auto ph_c, int s) {
    constexpr int PH = decltype(ph_c)::value;  // s mod U
    constexpr int CUR = PH % NR;                // ring slot consumed now
    load_row(P0 + s + PF, ring[(PH + PF) % NR]);
    if constexpr (GH) {
      const bool zg = P0 + s < 0 || P0 + s >= n_axis;
#pragma unroll
      for (int j = 0; j < VX; ++j) ring[CUR][j] = keep && !zg ? ring[CUR][j] : A(0);
    }
    unroll_seq(
        [&](auto li) {
          constexpr int l = KL - decltype(li)::value;  // deepest first
          const int e = s - (l - 1) * (R + 1);
          if (!(e >= (l - 1) * R && e < span + (2 * KL - l + 1) * R)) return;
          constexpr int EP = pmod(PH - (l - 1) * (R + 1), W);
          const int q = P0 + e - R;
          A row[VX + 2 * R];
#pragma unroll
          for (int j = 0; j < VX; ++j) row[R + j] = l == 1 ? ring[CUR][j] : done[l - 1][j];
#pragma unroll
          for (int k = 1; k <= R; ++k) {
            const int sh = (k + VX - 1) / VX;
            const A lv = row[R + VX * sh - k], rv = row[R + k - 1 - VX * (sh - 1)];
            row[R - k] = sh == 1 ? dpp_f<kDppWaveShr1>(lv) : dpp_f<kDppWaveShr1>(dpp_f<kDppWaveShr1>(lv));
            row[R + VX - 1 + k] =
                sh == 1 ? dpp_f<kDppWaveShl1>(rv) : dpp_f<kDppWaveShl1>(dpp_f<kDppWaveShl1>(rv));
          }
          A res[VX];
#pragma unroll
          for (int j = 0; j < VX; ++j) {
#pragma unroll
            for (int dz = -R; dz <= R; ++dz) {
              const int slot = ROT ? R + dz : pmod(EP - dz, W);
              A sum = dz == -R ? A(0) : acc[l - 1][j][slot];
#pragma unroll
              for (int dx = -R; dx <= R; ++dx) {
                const int wi = S::table.idx[dz + R][0][dx + R];
                if (wi >= 0) sum = fma_(a.w.w[wi], row[R + j + dx], sum);
              }
              acc[l - 1][j][slot] = sum;
            }
            const A v = acc[l - 1][j][ROT ? 2 * R : pmod(EP - R, W)];
            res[j] = RAS && l < KL ? v : Store<T>::round(v);
            if constexpr (ROT) {  // output e - R is done: every sum moves one slot up
#pragma unroll
              for (int k = 2 * R; k > 0; --k) acc[l - 1][j][k] = acc[l - 1][j][k - 1];
            }
          }
          if constexpr (GH) {
            const bool zg = q < 0 || q >= n_axis;
#pragma unroll
            for (int j = 0; j < VX; ++j) res[j] = keep && !zg ? res[j] : A(0);
          }
          if constexpr (l < KL) {
#pragma unroll
            for (int j = 0; j < VX; ++j) done[l][j] = res[j];
          } else if (st && q >= zo0 && q < zo1) {
            char *dst = reinterpret_cast<char *>(out + (int64_t)(q - (int)a.out_z0) * a.plane);
            VecIO<T, VX>::store(reinterpret_cast<T *>(dst + boff), res);
          }
        },
        std::make_integer_sequence<int, KL>{});
  };
  for (int s = 0; s < n_steps; s += U)
    unroll_seq([&](auto ph) { step(ph, s + decltype(ph)::value); }, std::make_integer_sequence<int, U>{});
}

// 4 independent waves per workgroup; wave task = (tile, segment).  RAS (round
// at store): levels below the last keep FP32 sums; only the value a launch
// stores is rounded to the storage type.
template <typename T, bool BOX, int R, int KL, int VX, int PF, bool ROT, bool RAS = false>
__global__ __launch_bounds__(256) void march2d_kernel(const TbArgs<typename Store<T>::A> a) {
  using G = RowTile<R, KL, VX>;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntask = a.ntx * a.nseg;
  const int wg = xcd_tile(blockIdx.x, (ntask + 3) / 4);
  if (wg < 0) return;
  const int task = wg * 4 + wave;
  if (task >= ntask) return;
  const int tx_i = task % a.ntx, seg = task / a.ntx;
  const int zo0 = (int)a.out_lo + seg * (int)a.zseg;
  if (zo0 >= (int)a.out_hi) return;
  const int zo1 = min(zo0 + (int)a.zseg, (int)a.out_hi);
  const int x_lo = tx_i * G::OX - G::HX;
  const int P0 = zo0 - KL * R, n_load = zo1 - zo0 + 2 * KL * R;
  const bool ghosts = (!a.per_x && (x_lo < 0 || x_lo + G::TX > a.nx)) || P0 - 2 * R < 0 ||
                      P0 + n_load + R > (int)a.n_axis;
  if (ghosts)
    march2d_tile<T, BOX, R, KL, VX, PF, ROT, RAS, true>(a, lane, tx_i, zo0, zo1);
  else
    march2d_tile<T, BOX, R, KL, VX, PF, ROT, RAS, false>(a, lane, tx_i, zo0, zo1);
}

}  // namespace so2dr
