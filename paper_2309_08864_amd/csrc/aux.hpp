// aux.hpp -- FP64 reductions used by the adjoint: the loss pass and the
// weight-gradient sums, each a fixed-order two-pass reduction (per-workgroup
// partials, then one in-order sum), so results do not depend on timing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace so2dr {

constexpr int kRedWgs = 1024;    // workgroups of a first reduction pass
constexpr int kMaxRedPts = 81;   // most stencil points (2D box of radius 4)

struct RedOffsets {
  int8_t dz[kMaxRedPts], dy[kMaxRedPts], dx[kMaxRedPts];
};

// lam_u: on entry u_T, on exit lambda_T = u_T - y (storage type), over n
// elements; adds 0.5 sum (u - y)^2 (FP64) to acc[0].
int launch_loss(int dtype, void *lam_u, const void *y, int64_t n, double *partials, double *acc,
                hipStream_t s);

// acc[k] += sum over planes [z0, z1) of lam(x) * ext(u, x + o_k), FP64.
// lam and u are slot buffers whose index 0 holds global plane buf_z0; planes
// outside [0, n_axis) are zero; in-plane axes wrap when periodic.
int launch_wgrad(int dtype, const void *lam, const void *u, int64_t buf_z0, int nx, int ny,
                 int per_x, int per_y, int64_t n_axis, int64_t z0, int64_t z1,
                 const RedOffsets &offs, int npts, double *partials, double *acc, hipStream_t s);

// dst <- src, `bytes` bytes of device-addressable memory, by a copy kernel
// of `grid` workgroups on stream s.
int launch_dcopy(void *dst, const void *src, size_t bytes, hipStream_t s, int grid = 1024);

}  // namespace so2dr
