// launch.hpp -- host-side description of one fused-step kernel launch and the
// per-storage-type dispatchers that map it onto a compiled instantiation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

namespace so2dr {

// Stencils with compiled kernels.  ndim/shape/radius -> id.
enum StencilId {
  ST_2D_STAR_R1 = 0,
  ST_2D_BOX_R1 = 1,
  ST_2D_BOX_R2 = 2,
  ST_2D_BOX_R3 = 3,
  ST_2D_BOX_R4 = 4,
  ST_3D_STAR_R1 = 5,
  ST_3D_STAR_R2 = 6,
  ST_3D_BOX_R1 = 7,
  ST_COUNT = 8
};

struct LaunchParams {
  int stencil;             // StencilId
  int kl;                  // fused levels
  const void *in;
  void *out;
  int64_t buf_z0, out_z0, plane;   // global planes at index 0 of in and out
  int nx, ny, per_x, per_y;
  int64_t n_axis, in_lo, in_hi, out_lo, out_hi;
  const double *weights;   // npts, lexicographic
  int npts;
  int ras = 0;             // 16-bit storage: round only what a launch stores
};

// Deepest compiled depth per storage type (so2dr_dtype) and stencil; 0 = none.
int max_depth(int dtype, int stencil);

// Launch on `stream`; returns 0 or a negative so2dr error code (msg filled).
int launch_tb(int dtype, const LaunchParams &p, hipStream_t stream, std::string *msg);

// Per-type entry points defined in kernels_<type>.hip.
int launch_tb_f32(const LaunchParams &p, hipStream_t s, std::string *msg);
int launch_tb_f64(const LaunchParams &p, hipStream_t s, std::string *msg);
int launch_tb_bf16(const LaunchParams &p, hipStream_t s, std::string *msg);
int launch_tb_f16(const LaunchParams &p, hipStream_t s, std::string *msg);

}  // namespace so2dr
