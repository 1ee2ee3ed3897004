// Setup-time kernels of the general path (element and patch diagonals, storage
// conversions) and the dense coarse solve.
#include <hip/hip_runtime.h>

#include "hex_launch.h"
#include "launch.h"

namespace pmg {

namespace {

template <int DIM>
__global__ __launch_bounds__(256) void k_cell_diag(int q, long total, const double *B, const double *Dn,
                                                   const double *G, double *out) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t < total) cell_diag<DIM, double>(t, q, B, Dn, G, out);
}

template <int DIM, typename S>
__global__ __launch_bounds__(256) void k_patch_invdiag(int q, int n, double omega, long total, const double *cdiag,
                                                       S *out) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t < total) patch_inv_diag<DIM, S>(t, q, n, omega, cdiag, out);
}

template <int DIM, typename S>
__global__ __launch_bounds__(256) void k_patch_invdiag_list(int q, double omega, long total, const int32_t *pcells,
                                                            const double *cdiag, S *out) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t < total) patch_inv_diag_list<DIM, S>(t, q, pcells, omega, cdiag, out);
}

__global__ __launch_bounds__(256) void k_identity(double *A, int m) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < m) A[i * m + i] = 1.0;
}

template <typename S>
__global__ __launch_bounds__(256) void k_convert(const double *in, S *out, long n) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = to_storage<S>(in[i]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_gather(int dim, int mi, int mt, const T *r, T *z, double *w) {
  const long tot = dim == 3 ? (long)mt * mt * mt : (long)mt * mt;
  for (long g = (long)blockIdx.x * 256 + threadIdx.x; g < tot; g += (long)gridDim.x * 256) {
    const int i = (int)(g % mt), j = (int)((g / mt) % mt), k = dim == 3 ? (int)(g / ((long)mt * mt)) : 1;
    const bool bnd = i == 0 || i == mt - 1 || j == 0 || j == mt - 1 || k == 0 || k == mt - 1;
    if (bnd) {
      z[g] = r[g];
    } else {
      const long e = (i - 1) + (long)mi * ((j - 1) + (long)mi * (dim == 3 ? k - 1 : 0));
      w[e] = (double)r[g];
    }
  }
}

// one wave per row of Ainv (m x m, symmetric): z_int[row] = sum_j Ainv[row][j] w[j]
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_gemv(int dim, int mi, int mt, long m, const double *Ainv,
                                                     const double *w, T *z) {
  const long row = (long)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= m) return;
  double s = 0.0;
  const double *a = Ainv + row * m;
  for (long j = lane; j < m; j += 64) s += a[j] * w[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) {
    const int i = (int)(row % mi), j = (int)((row / mi) % mi), k = dim == 3 ? (int)(row / ((long)mi * mi)) : 0;
    const long g = (i + 1) + (long)mt * ((j + 1) + (long)mt * (dim == 3 ? k + 1 : 0));
    z[g] = (T)s;
  }
}

int ok() { return hipGetLastError() == hipSuccess ? 0 : -4; }

}  // namespace

int launch_cell_diag(int dim, int q, long n_cells, const double *B, const double *Dn, const double *G, double *cdiag,
                     hipStream_t s) {
  const long kd = dim == 3 ? (long)(q + 1) * (q + 1) * (q + 1) : (long)(q + 1) * (q + 1);
  const long total = n_cells * kd;
  const unsigned grid = (unsigned)((total + 255) / 256);
  if (dim == 3)
    hipLaunchKernelGGL(k_cell_diag<3>, dim3(grid), dim3(256), 0, s, q, total, B, Dn, G, cdiag);
  else
    hipLaunchKernelGGL(k_cell_diag<2>, dim3(grid), dim3(256), 0, s, q, total, B, Dn, G, cdiag);
  return ok();
}

template <typename S>
int launch_patch_invdiag(int dim, int q, int n, double omega, const double *cdiag, S *invD, hipStream_t s) {
  const long e1 = 2 * q - 1, k1 = n - 1;
  const long total = dim == 3 ? k1 * k1 * k1 * e1 * e1 * e1 : k1 * k1 * e1 * e1;
  const unsigned grid = (unsigned)((total + 255) / 256);
  if (total == 0) return 0;
  if (dim == 3)
    hipLaunchKernelGGL((k_patch_invdiag<3, S>), dim3(grid), dim3(256), 0, s, q, n, omega, total, cdiag, invD);
  else
    hipLaunchKernelGGL((k_patch_invdiag<2, S>), dim3(grid), dim3(256), 0, s, q, n, omega, total, cdiag, invD);
  return ok();
}

template <typename S>
int launch_patch_invdiag_list(int dim, int q, long np, const int32_t *pcells, double omega, const double *cdiag,
                              S *invD, hipStream_t s) {
  const long e1 = 2 * q - 1;
  const long total = dim == 3 ? np * e1 * e1 * e1 : np * e1 * e1;
  if (total == 0) return 0;
  const unsigned grid = (unsigned)((total + 255) / 256);
  if (dim == 3)
    hipLaunchKernelGGL((k_patch_invdiag_list<3, S>), dim3(grid), dim3(256), 0, s, q, omega, total, pcells, cdiag, invD);
  else
    hipLaunchKernelGGL((k_patch_invdiag_list<2, S>), dim3(grid), dim3(256), 0, s, q, omega, total, pcells, cdiag, invD);
  return ok();
}

int launch_set_identity(double *A, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_identity, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, A, m);
  return ok();
}

template <typename S>
int launch_convert(const double *in, S *out, long n, hipStream_t s) {
  if (n == 0) return 0;
  hipLaunchKernelGGL((k_convert<S>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, n);
  return ok();
}

template <typename T>
int launch_coarse_dense(int dim, int mi, int mt, const double *Ainv, const T *r, T *z, double *w, hipStream_t s) {
  const long m = dim == 3 ? (long)mi * mi * mi : (long)mi * mi;
  hipLaunchKernelGGL((k_coarse_gather<T>), dim3(64), dim3(256), 0, s, dim, mi, mt, r, z, w);
  if (hipGetLastError() != hipSuccess) return -4;
  hipLaunchKernelGGL((k_coarse_gemv<T>), dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, dim, mi, mt, m, Ainv, w, z);
  return ok();
}

template int launch_patch_invdiag<double>(int, int, int, double, const double *, double *, hipStream_t);
template int launch_patch_invdiag<float>(int, int, int, double, const double *, float *, hipStream_t);
template int launch_patch_invdiag<bf16>(int, int, int, double, const double *, bf16 *, hipStream_t);
template int launch_patch_invdiag_list<double>(int, int, long, const int32_t *, double, const double *, double *,
                                               hipStream_t);
template int launch_patch_invdiag_list<float>(int, int, long, const int32_t *, double, const double *, float *,
                                              hipStream_t);
template int launch_convert<float>(const double *, float *, long, hipStream_t);
template int launch_convert<bf16>(const double *, bf16 *, long, hipStream_t);
template int launch_coarse_dense<double>(int, int, int, const double *, const double *, double *, double *,
                                         hipStream_t);
template int launch_coarse_dense<float>(int, int, int, const double *, const float *, float *, double *, hipStream_t);

}  // namespace pmg
