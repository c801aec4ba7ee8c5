// launch_impl.hpp -- shared by the kernels_<type>.hip files: builds the
// argument block, sizes the grid and launches one tb_kernel instantiation.
#pragma once
#include <algorithm>
#include <string>

#include "launch.hpp"
#include "tb_kernel.hpp"

namespace so2dr {

// Workgroups a launch aims for before it splits the cut axis into segments;
// each segment re-reads 2*KL*R input planes, so segments stay long.
#ifndef SO2DR_TARGET_WGS
#define SO2DR_TARGET_WGS 1024
#endif
#ifndef SO2DR_MIN_SEG
#define SO2DR_MIN_SEG 16
#endif
constexpr int64_t kTargetWgs = SO2DR_TARGET_WGS;
constexpr int64_t kMinSegPlanes = SO2DR_MIN_SEG;

template <typename T, int NDIM, bool BOX, int R, int KL>
int launch_one(const LaunchParams &p, hipStream_t stream, std::string *msg) {
  using A = typename Store<T>::A;
  using G = Tile<NDIM, R, KL>;
  using S = Stencil<NDIM, BOX, R>;
  if (p.npts != S::npts()) {
    if (msg) *msg = "weight count does not match the stencil";
    return -1;
  }
  TbArgs<A> a{};
  a.in = p.in;
  a.out = p.out;
  a.buf_z0 = p.buf_z0;
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
  for (int i = 0; i < S::npts(); ++i) a.w.w[i] = (A)p.weights[i];
  a.ntx = (int)((p.nx + G::OX - 1) / G::OX);
  a.nty = NDIM == 2 ? 1 : (int)((p.ny + G::OY - 1) / G::OY);
  const int64_t span = p.out_hi - p.out_lo;
  if (span <= 0) return 0;
  const int64_t tiles = (int64_t)a.ntx * a.nty;
  int64_t nseg = std::max<int64_t>(1, (kTargetWgs + tiles - 1) / tiles);
  nseg = std::min<int64_t>(nseg, std::max<int64_t>(1, span / kMinSegPlanes));
  a.zseg = (span + nseg - 1) / nseg;
  a.nseg = (int)((span + a.zseg - 1) / a.zseg);
  const int64_t nwg = tiles * a.nseg;
  if (nwg > 0x7fffffff) {
    if (msg) *msg = "grid too large for one launch";
    return -1;
  }
  constexpr size_t lds = tb_lds_bytes<T, NDIM, BOX, R, KL>();
  static bool attr_done = false;
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute((const void *)tb_kernel<T, NDIM, BOX, R, KL>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
      if (msg) *msg = std::string("hipFuncSetAttribute: ") + hipGetErrorString(e);
      return -5;
    }
    attr_done = true;
  }
  // with the XCD-aware order the grid is padded to a multiple of 8 so that the
  // permutation covers every tile; padding workgroups exit at once
  const int64_t grid = SO2DR_XCD_REMAP ? (nwg + 7) / 8 * 8 : nwg;
  hipLaunchKernelGGL((tb_kernel<T, NDIM, BOX, R, KL>), dim3((unsigned)grid), dim3(G::NT), lds, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (msg) *msg = std::string("kernel launch: ") + hipGetErrorString(e);
    return -5;
  }
  return 0;
}

// Expand one stencil's depths 1..MAXKL into a switch on p.kl.
template <typename T, int NDIM, bool BOX, int R, int MAXKL>
int launch_depth(const LaunchParams &p, hipStream_t s, std::string *msg) {
  switch (p.kl) {
    case 1: return launch_one<T, NDIM, BOX, R, 1>(p, s, msg);
    case 2: if constexpr (MAXKL >= 2) return launch_one<T, NDIM, BOX, R, 2>(p, s, msg); else break;
    case 3: if constexpr (MAXKL >= 3) return launch_one<T, NDIM, BOX, R, 3>(p, s, msg); else break;
    case 4: if constexpr (MAXKL >= 4) return launch_one<T, NDIM, BOX, R, 4>(p, s, msg); else break;
    case 5: if constexpr (MAXKL >= 5) return launch_one<T, NDIM, BOX, R, 5>(p, s, msg); else break;
    case 6: if constexpr (MAXKL >= 6) return launch_one<T, NDIM, BOX, R, 6>(p, s, msg); else break;
    case 7: if constexpr (MAXKL >= 7) return launch_one<T, NDIM, BOX, R, 7>(p, s, msg); else break;
    case 8: if constexpr (MAXKL >= 8) return launch_one<T, NDIM, BOX, R, 8>(p, s, msg); else break;
    default: break;
  }
  if (msg) *msg = "fused depth not built for this stencil";
  return -3;
}

}  // namespace so2dr
