// kernels.hip -- the fused-step kernels of one storage type, and the
// dispatcher that maps a launch onto a compiled instantiation.  The build
// compiles this file once per storage type, with SO2DR_STORAGE set to its
// so2dr_dtype value (0 F32, 1 F64, 2 BF16, 3 F16), so that the four sets of
// instantiations compile in parallel; kMaxDepth (depths.hpp) decides which
// stencils and depths each type gets.
#include "so2dr.h"

#include "depths.hpp"
#include "launch_impl.hpp"

#ifndef SO2DR_STORAGE
#error "compile with -DSO2DR_STORAGE=<so2dr_dtype value>"
#endif

namespace so2dr {
namespace {

template <int D> struct StorageOf;
template <> struct StorageOf<SO2DR_F32> { using T = float; };
template <> struct StorageOf<SO2DR_F64> { using T = double; };
template <> struct StorageOf<SO2DR_BF16> { using T = __hip_bfloat16; };
template <> struct StorageOf<SO2DR_F16> { using T = __half; };

template <int D>
int dispatch(const LaunchParams &p, hipStream_t s, std::string *msg) {
  using T = typename StorageOf<D>::T;
  switch (p.stencil) {
#define SO2DR_CASE(ID, NDIM, BOX, R)                                          \
  case ID:                                                                  \
    if constexpr (kMaxDepth[D][ID] > 0)                                     \
      return launch_depth<T, NDIM, BOX, R, kMaxDepth[D][ID]>(p, s, msg);   \
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

}  // namespace

#if SO2DR_STORAGE == 0
int launch_tb_f32(const LaunchParams &p, hipStream_t s, std::string *msg) { return dispatch<SO2DR_F32>(p, s, msg); }
#elif SO2DR_STORAGE == 1
int launch_tb_f64(const LaunchParams &p, hipStream_t s, std::string *msg) { return dispatch<SO2DR_F64>(p, s, msg); }
#elif SO2DR_STORAGE == 2
int launch_tb_bf16(const LaunchParams &p, hipStream_t s, std::string *msg) { return dispatch<SO2DR_BF16>(p, s, msg); }
#elif SO2DR_STORAGE == 3
int launch_tb_f16(const LaunchParams &p, hipStream_t s, std::string *msg) { return dispatch<SO2DR_F16>(p, s, msg); }
#else
#error "SO2DR_STORAGE must be 0, 1, 2 or 3"
#endif

}  // namespace so2dr
