// aux_kernels.hip -- FP64 reductions of the adjoint (loss and weight
// gradients).  Not in the paper: the gradient of L = 1/2 ||u_T - y||^2 with
// respect to the weights is sum_t sum_x lambda_{t+1}(x) u_t(x + o_k), and the
// loss itself; both are accumulated in FP64 on the GPU.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "aux.hpp"
#include "../../include/so2dr.h"

namespace so2dr {

constexpr int kRedThreads = 256;

template <typename T>
__device__ __forceinline__ double to_d(T v) { return (double)v; }

__device__ __forceinline__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Device-to-device copy on the caller's stream, by a kernel of our own (the
// region-sharing copies): 16-byte accesses where both ends allow, else 4 or 1.
template <typename W>
__global__ __launch_bounds__(256) void dcopy_kernel(W *__restrict__ dst, const W *__restrict__ src, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

int launch_dcopy(void *dst, const void *src, size_t bytes, hipStream_t s, int grid) {
  if (bytes == 0) return 0;
  const uintptr_t a = (uintptr_t)dst | (uintptr_t)src;
  grid = grid < 1 ? 1 : grid;
  if (a % 16 == 0 && bytes % 16 == 0) {
    hipLaunchKernelGGL(dcopy_kernel<uint4>, dim3(grid), dim3(256), 0, s, static_cast<uint4 *>(dst),
                       static_cast<const uint4 *>(src), (int64_t)(bytes / 16));
  } else if (a % 4 == 0 && bytes % 4 == 0) {
    hipLaunchKernelGGL(dcopy_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, static_cast<uint32_t *>(dst),
                       static_cast<const uint32_t *>(src), (int64_t)(bytes / 4));
  } else {
    hipLaunchKernelGGL(dcopy_kernel<uint8_t>, dim3(grid), dim3(256), 0, s, static_cast<uint8_t *>(dst),
                       static_cast<const uint8_t *>(src), (int64_t)bytes);
  }
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

template <typename T>
__global__ __launch_bounds__(256) void loss_kernel(T *lam_u, const T *y, int64_t n, double *partials) {
  __shared__ double red[kRedThreads];
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double d = to_d(lam_u[i]) - to_d(y[i]);   // exact for FP32 inputs
    lam_u[i] = (T)d;                                 // one rounding, as u - y in T
    s += 0.5 * d * d;
  }
  const double b = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

// acc[k] += sum_b partials[b * np + k]: one workgroup per k; lane t sums
// b = t, t + 256, ... in order, then a fixed tree -- the same order every run.
__global__ __launch_bounds__(256) void reduce_partials(const double *partials, int nb, int np, double *acc) {
  __shared__ double red[kRedThreads];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads) s += partials[(int64_t)b * np + k];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) acc[k] += t;
}

// Per workgroup, partials[block * NP + k] = sum over its cells x of
// lam(x) u(x + o_k).  Workgroups take whole rows of the owned planes in turn
// (row index -> plane and y once per row, uniform), lanes stride along x, so
// loads are coalesced and no per-cell division is needed.  A lane loads the
// values of up to 4 cells of its row (x, x + 256, ...) before it accumulates any,
// so each wave keeps several cells' loads in flight instead of one's; the
// accumulation order per lane is unchanged (cells by increasing x, points in
// order), and neighbours outside the grid are loaded from a clamped in-grid
// address and not accumulated.
template <typename T, int NP>
__global__ __launch_bounds__(256) void wgrad_kernel(const T *lam, const T *u, int64_t buf_z0, int nx,
                                                    int ny, int per_x, int per_y, int64_t n_axis,
                                                    int64_t z0, int64_t z1, RedOffsets o,
                                                    double *partials) {
  constexpr int WU = NP <= 13 ? 4 : NP <= 27 ? 2 : 1;  // cells per lane in flight
  __shared__ double red[kRedThreads];
  double acc[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) acc[k] = 0.0;
  const int64_t plane = (int64_t)nx * ny;
  const int64_t nrows = (z1 - z0) * ny;
  for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
    const int64_t z = z0 + row / ny;
    const int y = (int)(row % ny);
    const T *lrow = lam + (z - buf_z0) * plane + (int64_t)y * nx;
    // per point: its row of u (clamped into the grid) and whether that row exists
    const T *urow[NP];
    bool row_ok[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      int64_t zz = z + o.dz[k];
      int yy = y + o.dy[k];
      bool ok = zz >= 0 && zz < n_axis;
      if (yy < 0 || yy >= ny) {
        if (per_y) yy = yy < 0 ? yy + ny : yy - ny; else ok = false;
      }
      zz = ok ? zz : z;
      yy = ok ? yy : y;
      urow[k] = u + (zz - buf_z0) * plane + (int64_t)yy * nx;
      row_ok[k] = ok;
    }
    for (int xb = 0; xb < nx; xb += 256 * WU) {
      T l[WU];
      T v[WU][NP];
      bool use[WU][NP];
#pragma unroll
      for (int j = 0; j < WU; ++j) {
        const int x = xb + threadIdx.x + 256 * j;
        const bool in = x < nx;
        l[j] = lrow[in ? x : 0];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          int xx = x + o.dx[k];
          bool ok = in && row_ok[k];
          if (xx < 0 || xx >= nx) {
            if (per_x) xx = xx < 0 ? xx + nx : xx - nx; else ok = false;
          }
          xx = ok ? xx : 0;
          v[j][k] = urow[k][xx];
          use[j][k] = ok;
        }
      }
#pragma unroll
      for (int j = 0; j < WU; ++j)
#pragma unroll
        for (int k = 0; k < NP; ++k)
          if (use[j][k]) acc[k] += to_d(l[j]) * to_d(v[j][k]);
    }
  }
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double b = block_sum(acc[k], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * NP + k] = b;
  }
}

template <typename T>
static int loss_t(void *lam_u, const void *y, int64_t n, double *partials, double *acc, hipStream_t s) {
  hipLaunchKernelGGL(loss_kernel<T>, dim3(kRedWgs), dim3(kRedThreads), 0, s, static_cast<T *>(lam_u),
                     static_cast<const T *>(y), n, partials);
  hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kRedThreads), 0, s, partials, kRedWgs, 1, acc);
  return hipGetLastError() == hipSuccess ? 0 : SO2DR_E_HIP;
}

int launch_loss(int dtype, void *lam_u, const void *y, int64_t n, double *partials, double *acc,
                hipStream_t s) {
  if (n <= 0) return 0;
  switch (dtype) {
    case SO2DR_F32: return loss_t<float>(lam_u, y, n, partials, acc, s);
    case SO2DR_F64: return loss_t<double>(lam_u, y, n, partials, acc, s);
    default: return SO2DR_E_UNSUPPORTED;
  }
}

template <typename T, int NP>
static int wgrad_np(const void *lam, const void *u, int64_t buf_z0, int nx, int ny, int per_x, int per_y,
                    int64_t n_axis, int64_t z0, int64_t z1, const RedOffsets &o, double *partials,
                    double *acc, hipStream_t s) {
  hipLaunchKernelGGL((wgrad_kernel<T, NP>), dim3(kRedWgs), dim3(kRedThreads), 0, s,
                     static_cast<const T *>(lam), static_cast<const T *>(u), buf_z0, nx, ny, per_x,
                     per_y, n_axis, z0, z1, o, partials);
  hipLaunchKernelGGL(reduce_partials, dim3(NP), dim3(kRedThreads), 0, s, partials, kRedWgs, NP, acc);
  return hipGetLastError() == hipSuccess ? 0 : SO2DR_E_HIP;
}

template <typename T>
static int wgrad_t(const void *lam, const void *u, int64_t buf_z0, int nx, int ny, int per_x, int per_y,
                   int64_t n_axis, int64_t z0, int64_t z1, const RedOffsets &o, int npts,
                   double *partials, double *acc, hipStream_t s) {
#define SO2DR_NP(N) \
  case N: return wgrad_np<T, N>(lam, u, buf_z0, nx, ny, per_x, per_y, n_axis, z0, z1, o, partials, acc, s);
  switch (npts) {
    SO2DR_NP(5) SO2DR_NP(7) SO2DR_NP(9) SO2DR_NP(13) SO2DR_NP(25) SO2DR_NP(27) SO2DR_NP(49) SO2DR_NP(81)
    default: return SO2DR_E_UNSUPPORTED;
  }
#undef SO2DR_NP
}

int launch_wgrad(int dtype, const void *lam, const void *u, int64_t buf_z0, int nx, int ny, int per_x,
                 int per_y, int64_t n_axis, int64_t z0, int64_t z1, const RedOffsets &offs, int npts,
                 double *partials, double *acc, hipStream_t s) {
  if (z1 <= z0) return 0;
  switch (dtype) {
    case SO2DR_F32:
      return wgrad_t<float>(lam, u, buf_z0, nx, ny, per_x, per_y, n_axis, z0, z1, offs, npts, partials, acc, s);
    case SO2DR_F64:
      return wgrad_t<double>(lam, u, buf_z0, nx, ny, per_x, per_y, n_axis, z0, z1, offs, npts, partials, acc, s);
    default:
      return SO2DR_E_UNSUPPORTED;
  }
}

}  // namespace so2dr
