// kernels_f64.hip -- compiled fused-step kernels for double storage.
#include "depths.hpp"
#include "launch_impl.hpp"

namespace so2dr {

using T_f64 = double;

int launch_tb_f64(const LaunchParams &p, hipStream_t s, std::string *msg) {
  constexpr int D = 1;
  switch (p.stencil) {
#define SO2DR_CASE(ID, NDIM, BOX, R)                                                  \
  case ID:                                                                          \
    if constexpr (kMaxDepth[D][ID] > 0)                                             \
      return launch_depth<T_f64, NDIM, BOX, R, kMaxDepth[D][ID]>(p, s, msg);       \
    break;
    SO2DR_CASE(ST_2D_STAR_R1, 2, false, 1)
    SO2DR_CASE(ST_2D_BOX_R1, 2, true, 1)
    SO2DR_CASE(ST_2D_BOX_R2, 2, true, 2)
    SO2DR_CASE(ST_2D_BOX_R3, 2, true, 3)
    SO2DR_CASE(ST_2D_BOX_R4, 2, true, 4)
    SO2DR_CASE(ST_3D_STAR_R1, 3, false, 1)
    SO2DR_CASE(ST_3D_STAR_R2, 3, false, 2)
    SO2DR_CASE(ST_3D_BOX_R1, 3, true, 1)
#undef SO2DR_CASE
    default:
      break;
  }
  if (msg) *msg = "stencil not built for this storage type";
  return -3;
}

}  // namespace so2dr
