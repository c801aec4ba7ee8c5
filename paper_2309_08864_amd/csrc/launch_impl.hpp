// launch_impl.hpp -- shared by the kernels_<type>.hip files: builds the
// argument block, sizes the grid and launches one tb_kernel instantiation.
#pragma once
#include <atomic>
#include <algorithm>
#include <string>

#include "launch.hpp"
#include "march2d_kernel.hpp"
#include "march_kernel.hpp"
#include "star_kernel.hpp"
#include "tb_kernel.hpp"

namespace so2dr {

// Workgroups a launch aims for before it splits the cut axis into segments;
// each segment re-reads 2*KL*R input planes, so segments stay long.
constexpr int64_t kTargetWgs = 1024;
constexpr int64_t kMinSegPlanes = 16;

// Segmenting of the cut axis shared by both kernel families: `target`
// workgroups, never segments shorter than kMinSegPlanes.
inline void plan_segments(int64_t span, int64_t tiles, int64_t *zseg, int *nseg,
                          int64_t target = kTargetWgs) {
  int64_t n = std::max<int64_t>(1, (target + tiles - 1) / tiles);
  n = std::min<int64_t>(n, std::max<int64_t>(1, span / kMinSegPlanes));
  *zseg = (span + n - 1) / n;
  *nseg = (int)((span + *zseg - 1) / *zseg);
}

// Workgroups of `kernel` (block of `threads`) that the current device holds
// at once: resident workgroups per CU times CUs; 0 if the runtime cannot
// tell.  Per-CU residency depends only on the kernel, so it is asked once
// per kernel; the CU count once per device.
inline int64_t resident_wgs(const void *kernel, int threads, std::atomic<int> *per_cu_cache) {
  int per_cu = per_cu_cache->load(std::memory_order_relaxed);
  if (per_cu < 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess) per_cu = 0;
    per_cu_cache->store(per_cu, std::memory_order_relaxed);
  }
  static std::atomic<int> cu_count[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  int cus = cu_count[dev].load(std::memory_order_relaxed);
  if (cus <= 0) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
    cu_count[dev].store(cus, std::memory_order_relaxed);
  }
  return (int64_t)per_cu * cus;
}

// The argument block every kernel takes: buffers, geometry, planes and the
// weights converted to the accumulation type.  Tile counts and segmenting
// are the caller's.
template <typename A>
inline TbArgs<A> launch_args(const LaunchParams &p, int npts) {
  TbArgs<A> a{};
  a.in = p.in;
  a.out = p.out;
  a.buf_z0 = p.buf_z0;
  a.out_z0 = p.out_z0;
  a.plane = p.plane;
  a.nx = p.nx;
  a.ny = p.ny;
  a.per_x = p.per_x;
  a.per_y = p.per_y;
  a.n_axis = p.n_axis;
  a.in_lo = p.in_lo;
  a.in_hi = p.in_hi;
  a.out_lo = p.out_lo;
  a.out_hi = p.out_hi;
  for (int i = 0; i < npts; ++i) a.w.w[i] = (A)p.weights[i];
  return a;
}

template <typename T, int NDIM, bool BOX, int R, int KL, bool RAS = false>
int launch_one(const LaunchParams &p, hipStream_t stream, std::string *msg) {
  using A = typename Store<T>::A;
  using G = Tile<NDIM, R, KL>;
  using S = Stencil<NDIM, BOX, R>;
  if (p.npts != S::npts()) {
    if (msg) *msg = "weight count does not match the stencil";
    return -1;
  }
  TbArgs<A> a = launch_args<A>(p, S::npts());
  a.ntx = (int)((p.nx + G::OX - 1) / G::OX);
  a.nty = NDIM == 2 ? 1 : (int)((p.ny + G::OY - 1) / G::OY);
  const int64_t span = p.out_hi - p.out_lo;
  if (span <= 0) return 0;
  plan_segments(span, (int64_t)a.ntx * a.nty, &a.zseg, &a.nseg);
  const int64_t nwg = (int64_t)a.ntx * a.nty * a.nseg;
  if (nwg > 0x7fffffff) {
    if (msg) *msg = "grid too large for one launch";
    return -1;
  }
  constexpr size_t lds = tb_lds_bytes<T, NDIM, BOX, R, KL>();
  // once per instantiation; threads racing here both set the same value
  static std::atomic<bool> attr_done{false};
  if (!attr_done.load(std::memory_order_acquire)) {
    hipError_t e = hipFuncSetAttribute((const void *)tb_kernel<T, NDIM, BOX, R, KL, RAS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
      if (msg) *msg = std::string("hipFuncSetAttribute: ") + hipGetErrorString(e);
      return -5;
    }
    attr_done.store(true, std::memory_order_release);
  }
  const int64_t grid = xcd_grid(nwg);
  hipLaunchKernelGGL((tb_kernel<T, NDIM, BOX, R, KL, RAS>), dim3((unsigned)grid), dim3(G::NT), lds, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (msg) *msg = std::string("kernel launch: ") + hipGetErrorString(e);
    return -5;
  }
  return 0;
}

template <typename T, bool BOX, int R, int KL, int NW, int M, int VX, int HB, bool RAS = false>
int launch_col_one(const LaunchParams &p, hipStream_t stream, std::string *msg) {
  using A = typename Store<T>::A;
  using G = StarTile<R, KL, NW, M, VX>;
  using S = Stencil<3, BOX, R>;
  if (p.npts != S::npts()) {
    if (msg) *msg = "weight count does not match the stencil";
    return -1;
  }
  TbArgs<A> a = launch_args<A>(p, S::npts());
  a.ntx = (int)((p.nx + G::OX - 1) / G::OX);
  a.nty = (int)((p.ny + G::OY - 1) / G::OY);
  const int64_t span = p.out_hi - p.out_lo;
  if (span <= 0) return 0;
  plan_segments(span, (int64_t)a.ntx * a.nty, &a.zseg, &a.nseg);
  const int64_t nwg = (int64_t)a.ntx * a.nty * a.nseg;
  if (nwg > 0x7fffffff) {
    if (msg) *msg = "grid too large for one launch";
    return -1;
  }
  const int64_t grid = xcd_grid(nwg);
  hipLaunchKernelGGL((col3d_kernel<T, BOX, R, KL, NW, M, VX, HB, RAS>), dim3((unsigned)grid), dim3(NW * 64), 0,
                     stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (msg) *msg = std::string("kernel launch: ") + hipGetErrorString(e);
    return -5;
  }
  return 0;
}

// Whether the march kernel's layout fits this launch: whole VX-cell vectors
// per row, 32-bit byte offsets within a plane, 32-bit plane indices.
template <typename T, int VX>
inline bool march_fits(const LaunchParams &p) {
  // the kernels clamp loads into [max(in_lo, 0), min(in_hi, n_axis)): that
  // range must be non-empty
  return p.nx % VX == 0 && (uint64_t)p.plane * sizeof(T) < ((uint64_t)1 << 32) &&
         p.n_axis < ((int64_t)1 << 30) && p.in_lo > -((int64_t)1 << 29) && p.buf_z0 > -((int64_t)1 << 29) &&
         p.out_z0 > -((int64_t)1 << 29) && std::max<int64_t>(p.in_lo, 0) < std::min<int64_t>(p.in_hi, p.n_axis);
}

template <typename T, bool BOX, int R, int KL, int NW, int M, int VX, int HB, int PF, int WPE = 1,
          bool RAS = false, int HA = VX>
int launch_march_one(const LaunchParams &p, hipStream_t stream, std::string *msg) {
  using A = typename Store<T>::A;
  using G = StarTile<R, KL, NW, M, VX, HA>;
  using S = Stencil<3, BOX, R>;
  if (p.npts != S::npts()) {
    if (msg) *msg = "weight count does not match the stencil";
    return -1;
  }
  if (!march_fits<T, VX>(p)) {
    if (msg) *msg = "launch does not fit the march kernel's layout";
    return -1;
  }
  TbArgs<A> a = launch_args<A>(p, S::npts());
  a.ntx = (int)((p.nx + G::OX - 1) / G::OX);
  a.nty = (int)((p.ny + G::OY - 1) / G::OY);
  const int64_t span = p.out_hi - p.out_lo;
  if (span <= 0) return 0;
  // About 1.5 workgroups per resident slot: measured on MI355X over
  // 2048x1024x80 chunks, fewer leave the last wave of workgroups short and
  // more re-read 2 KL R planes per extra segment.
  static std::atomic<int> per_cu{-1};
  const void *kfn = (const void *)march3d_kernel<T, BOX, R, KL, NW, M, VX, HB, PF, WPE, RAS, HA>;
  const int64_t slots = resident_wgs(kfn, NW * 64, &per_cu);
  plan_segments(span, (int64_t)a.ntx * a.nty, &a.zseg, &a.nseg, slots > 0 ? slots * 3 / 2 : kTargetWgs);
  const int64_t nwg = (int64_t)a.ntx * a.nty * a.nseg;
  if (nwg > 0x7fffffff) {
    if (msg) *msg = "grid too large for one launch";
    return -1;
  }
  const int64_t grid = xcd_grid(nwg);
  hipLaunchKernelGGL((march3d_kernel<T, BOX, R, KL, NW, M, VX, HB, PF, WPE, RAS, HA>), dim3((unsigned)grid), dim3(NW * 64), 0,
                     stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (msg) *msg = std::string("kernel launch: ") + hipGetErrorString(e);
    return -5;
  }
  return 0;
}

template <typename T, bool BOX, int R, int KL, int VX, int PF, bool ROT, bool RAS = false>
int launch_march2d_one(const LaunchParams &p, hipStream_t stream, std::string *msg) {
  using A = typename Store<T>::A;
  using G = RowTile<R, KL, VX>;
  using S = Stencil<2, BOX, R>;
  if (p.npts != S::npts()) {
    if (msg) *msg = "weight count does not match the stencil";
    return -1;
  }
  if (!march_fits<T, VX>(p)) {
    if (msg) *msg = "launch does not fit the march kernel's layout";
    return -1;
  }
  TbArgs<A> a = launch_args<A>(p, S::npts());
  a.ntx = (int)((p.nx + G::OX - 1) / G::OX);
  a.nty = 1;
  const int64_t span = p.out_hi - p.out_lo;
  if (span <= 0) return 0;
  // one wave per (tile, segment); aim for 4 waves per targeted workgroup
  plan_segments(span, ((int64_t)a.ntx + 3) / 4, &a.zseg, &a.nseg);
  const int64_t tasks = (int64_t)a.ntx * a.nseg;
  const int64_t nwg = (tasks + 3) / 4;
  if (nwg > 0x7fffffff / 4) {
    if (msg) *msg = "grid too large for one launch";
    return -1;
  }
  const int64_t grid = xcd_grid(nwg);
  hipLaunchKernelGGL((march2d_kernel<T, BOX, R, KL, VX, PF, ROT, RAS>), dim3((unsigned)grid), dim3(256), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (msg) *msg = std::string("kernel launch: ") + hipGetErrorString(e);
    return -5;
  }
  return 0;
}

// Bytes of the march kernel's halo buffers.
template <typename A, int KL, int NW, int R, int VX, int HB>
constexpr size_t march_lds() {
  return sizeof(A) * KL * HB * NW * 2 * R * 64 * VX;
}

// Kernel choice per depth, from measurements on MI355X (one launch over a
// 2048x1024x80 FP32 chunk; all variants give identical bits):
//   * single-step launches run best with 1 KiB rows (4 cells per lane, 16
//     waves of 2 rows): 0.32 ms, 4.1 TB/s;
//   * two fused steps of the radius-1 star: 1 KiB rows, 8 waves of 4 rows
//     (0.28 ms, 4.6 TB/s);
//   * three fused steps of the radius-1 star and two of the radius-2 star:
//     512-byte rows, 8 waves of 6 rows (taller tiles re-read fewer halo rows;
//     1.37 and 0.82 T updates/s);
//   * other deeper fusion and the 27-point box: 512-byte rows, 8 waves of 4
//     rows (27-point at 2 levels 0.70 T updates/s);
//   (the taller shapes hold FP32 sums only: FP64 keeps the 4-row tiles)
//   * grids whose row length is not a multiple of the cells per lane fall
//     back to the register-column kernel, 2D grids and whatever does not fit
//     to the LDS-plane kernel.
template <typename T, int NDIM, bool BOX, int R, int KL, bool RAS>
int launch_any(const LaunchParams &p, hipStream_t s, std::string *msg) {
  using A = typename Store<T>::A;
  constexpr size_t kLdsMax = 160 * 1024;
  if constexpr (NDIM == 2) {
    // unrolling by the stencil width is kept while the unrolled body stays
    // within a few thousand FMAs
    constexpr bool rot = (int64_t)KL * 4 * Stencil<2, BOX, R>::npts() * (2 * R + 1) > 2400;
    if (march_fits<T, 4>(p)) return launch_march2d_one<T, BOX, R, KL, 4, 2, rot, RAS>(p, s, msg);
  }
  if constexpr (NDIM == 3) {
    constexpr bool wide = KL == 1 && march_lds<A, KL, 16, R, 4, 2>() <= kLdsMax;
    constexpr bool a32 = sizeof(A) == 4;
    constexpr bool square = a32 && !BOX && R == 1 && KL == 2;
    constexpr bool tall = a32 && !BOX && ((R == 1 && KL == 3) || (R == 2 && KL == 2));
    constexpr int HB = march_lds<A, KL, 8, R, 2, 2>() <= 65536 ? 2 : 1;
    // Star tiles of 1 KiB FP32 rows (2 KiB FP64) take a 64-byte x halo: each
    // output row is then whole 128-byte lines.  Measured on 2048x1024
    // planes: single-step launches 3-8 % faster (FP32 7- and 13-point, FP64)
    // and the two-step 7-point launch 0-3 % faster than with the 4-cell halo,
    // whose output rows share lines with the neighbouring tiles.  The
    // 512-byte-row shapes of deeper fusion and the 27-point box lose more to
    // the wider halo's arithmetic than they gain; 16-bit rows gain nothing.
    constexpr int HA4 = BOX ? 4 : sizeof(T) == 4 ? 16 : sizeof(T) == 8 ? 8 : 4;
    if constexpr (wide) {
      if (march_fits<T, 4>(p)) return launch_march_one<T, BOX, R, KL, 16, 2, 4, 2, 2, 1, RAS, HA4>(p, s, msg);
    } else {
      if constexpr (square)
        if (march_fits<T, 4>(p)) return launch_march_one<T, BOX, R, KL, 8, 4, 4, 2, 2, 1, RAS, HA4>(p, s, msg);
      if constexpr (tall)
        if (march_fits<T, 2>(p)) return launch_march_one<T, BOX, R, KL, 8, 6, 2, 2, 2, 1, RAS>(p, s, msg);
      if constexpr (march_lds<A, KL, 8, R, 2, HB>() <= kLdsMax && 2 * ((KL * R + 1) / 2) < 32 &&
                    4 >= R && 32 > 2 * KL * R)
        if (march_fits<T, 2>(p)) return launch_march_one<T, BOX, R, KL, 8, 4, 2, HB, 2, 1, RAS>(p, s, msg);
    }
  }
  constexpr size_t lds1 = sizeof(A) * KL * 1 * 16 * 2 * R * 64 * 4;
  constexpr size_t ldsn = sizeof(A) * KL * 2 * 4 * 2 * R * 64 * 1;
  if constexpr (NDIM == 3 && KL == 1 && lds1 <= 65536)
    return launch_col_one<T, BOX, R, KL, 16, 2, 4, 1, RAS>(p, s, msg);
  else if constexpr (NDIM == 3 && KL >= 2 && 2 * KL * R < 32 && ldsn <= 65536)
    return launch_col_one<T, BOX, R, KL, 4, 8, 1, 2, RAS>(p, s, msg);
  else
    return launch_one<T, NDIM, BOX, R, KL, RAS>(p, s, msg);
}

// Expand one stencil's depths 1..MAXKL into a switch on p.kl.
template <typename T, int NDIM, bool BOX, int R, int MAXKL, bool RAS>
int launch_depth_r(const LaunchParams &p, hipStream_t s, std::string *msg) {
  switch (p.kl) {
    case 1: return launch_any<T, NDIM, BOX, R, 1, RAS>(p, s, msg);
    case 2: if constexpr (MAXKL >= 2) return launch_any<T, NDIM, BOX, R, 2, RAS>(p, s, msg); else break;
    case 3: if constexpr (MAXKL >= 3) return launch_any<T, NDIM, BOX, R, 3, RAS>(p, s, msg); else break;
    case 4: if constexpr (MAXKL >= 4) return launch_any<T, NDIM, BOX, R, 4, RAS>(p, s, msg); else break;
    case 5: if constexpr (MAXKL >= 5) return launch_any<T, NDIM, BOX, R, 5, RAS>(p, s, msg); else break;
    case 6: if constexpr (MAXKL >= 6) return launch_any<T, NDIM, BOX, R, 6, RAS>(p, s, msg); else break;
    case 7: if constexpr (MAXKL >= 7) return launch_any<T, NDIM, BOX, R, 7, RAS>(p, s, msg); else break;
    case 8: if constexpr (MAXKL >= 8) return launch_any<T, NDIM, BOX, R, 8, RAS>(p, s, msg); else break;
    default: break;
  }
  if (msg) *msg = "fused depth not built for this stencil";
  return -3;
}

// Round-at-store variants exist for the 16-bit storage types only: FP32 and
// FP64 storage rounds nothing between levels either way.
template <typename T, int NDIM, bool BOX, int R, int MAXKL>
int launch_depth(const LaunchParams &p, hipStream_t s, std::string *msg) {
  if constexpr (sizeof(T) == 2) {
    if (p.ras) return launch_depth_r<T, NDIM, BOX, R, MAXKL, true>(p, s, msg);
  }
  return launch_depth_r<T, NDIM, BOX, R, MAXKL, false>(p, s, msg);
}

}  // namespace so2dr
