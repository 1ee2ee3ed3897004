// Vector kernels of the outer flexible CG: deterministic dot products (fixed grid, fixed
// reduction tree, so repeated runs give bitwise identical scalars), fused updates, casts.
#include <hip/hip_runtime.h>

#include <cmath>

#include "launch.h"

namespace pmg {

namespace {

constexpr int kThreads = 256;

__device__ inline double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kThreads) void k_dot_partial(const double *__restrict__ x, const double *__restrict__ y0,
                                                          const double *__restrict__ y1, long n,
                                                          double *__restrict__ part) {
  __shared__ double sh[kThreads];
  double s0 = 0.0, s1 = 0.0;
  const long stride = (long)gridDim.x * kThreads;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
    const double xi = x[i];
    s0 += xi * y0[i];
    if (y1) s1 += xi * y1[i];
  }
  s0 = block_sum(s0, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s0;
  if (y1) {
    s1 = block_sum(s1, sh);
    if (threadIdx.x == 0) part[kRedBlocks + blockIdx.x] = s1;
  }
}

__global__ __launch_bounds__(kThreads) void k_dot_final(const double *__restrict__ part, int ny, int mode, int i0,
                                                        double *__restrict__ scal) {
  __shared__ double sh[kThreads];
  double v[2] = {0.0, 0.0};
  for (int k = 0; k < ny; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kThreads) s += part[k * kRedBlocks + i];
    v[k] = block_sum(s, sh);
  }
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    scal[i0] = v[0];
  } else if (mode == 1) {
    scal[S_PQ] = v[0];
    scal[S_ALPHA] = scal[S_RZ] / v[0];
  } else {
    scal[S_ZRN] = v[0];
    scal[S_ZRO] = v[1];
    scal[S_BETA] = (v[0] - v[1]) / scal[S_RZ];
    scal[S_RZ] = v[0];
  }
}

__global__ __launch_bounds__(kThreads) void k_fcg_xr(double *__restrict__ x, const double *__restrict__ ro,
                                                     double *__restrict__ rn, const double *__restrict__ p,
                                                     const double *__restrict__ q, const double *__restrict__ scal,
                                                     long n, double *__restrict__ part) {
  __shared__ double sh[kThreads];
  const double alpha = scal[S_ALPHA];
  double s = 0.0;
  const long stride = (long)gridDim.x * kThreads;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
    x[i] += alpha * p[i];
    const double r = ro[i] - alpha * q[i];
    rn[i] = r;
    s += r * r;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void k_fcg_p(double *__restrict__ p, const double *__restrict__ z,
                                                    const double *__restrict__ scal, long n) {
  const double beta = scal[S_BETA];
  const long stride = (long)gridDim.x * kThreads;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) p[i] = z[i] + beta * p[i];
}

__global__ __launch_bounds__(kThreads) void k_copy(double *__restrict__ d, const double *__restrict__ s, long n) {
  const long stride = (long)gridDim.x * kThreads;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) d[i] = s[i];
}

__global__ __launch_bounds__(kThreads) void k_d2f(const double *__restrict__ in, float *__restrict__ out, long n) {
  const long stride = (long)gridDim.x * kThreads;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) out[i] = (float)in[i];
}

__global__ __launch_bounds__(kThreads) void k_f2d(const float *__restrict__ in, double *__restrict__ out, long n) {
  const long stride = (long)gridDim.x * kThreads;
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) out[i] = (double)in[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_init_z(int dim, int m, T *__restrict__ z, const T *__restrict__ r,
                                                     long n) {
  const long stride = (long)gridDim.x * kThreads;
  for (long g = (long)blockIdx.x * kThreads + threadIdx.x; g < n; g += stride) {
    const int i = (int)(g % m), j = (int)((g / m) % m), k = dim == 3 ? (int)(g / ((long)m * m)) : 1;
    const bool bnd = i == 0 || i == m - 1 || j == 0 || j == m - 1 || k == 0 || k == m - 1;
    z[g] = bnd ? r[g] : T(0);
  }
}

int grid_for(long n) {
  long g = (n + kThreads - 1) / kThreads;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

int ok() { return hipGetLastError() == hipSuccess ? 0 : -4; }

}  // namespace

int launch_dot_partial(const double *x, const double *y0, const double *y1, long n, double *partial, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(kThreads), 0, s, x, y0, y1, n, partial);
  return ok();
}

int launch_dot_final(const double *partial, int ny, int mode, int i0, double *scal, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kThreads), 0, s, partial, ny, mode, i0, scal);
  return ok();
}

int launch_fcg_xr(double *x, const double *ro, double *rn, const double *p, const double *q, const double *scal,
                  long n, double *partial, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_xr, dim3(kRedBlocks), dim3(kThreads), 0, s, x, ro, rn, p, q, scal, n, partial);
  return ok();
}

int launch_fcg_p(double *p, const double *z, const double *scal, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_p, dim3(grid_for(n)), dim3(kThreads), 0, s, p, z, scal, n);
  return ok();
}

int launch_copy(double *dst, const double *src, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(kThreads), 0, s, dst, src, n);
  return ok();
}

int launch_cast_d2f(const double *in, float *out, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_d2f, dim3(grid_for(n)), dim3(kThreads), 0, s, in, out, n);
  return ok();
}

int launch_cast_f2d(const float *in, double *out, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_f2d, dim3(grid_for(n)), dim3(kThreads), 0, s, in, out, n);
  return ok();
}

template <typename T>
int launch_init_z(int dim, int m, T *z, const T *r, hipStream_t s) {
  long n = dim == 3 ? (long)m * m * m : (long)m * m;
  hipLaunchKernelGGL((k_init_z<T>), dim3(grid_for(n)), dim3(kThreads), 0, s, dim, m, z, r, n);
  return ok();
}

template int launch_init_z<double>(int, int, double *, const double *, hipStream_t);
template int launch_init_z<float>(int, int, float *, const float *, hipStream_t);

}  // namespace pmg
