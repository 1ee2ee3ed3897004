// Host-side launchers of the HIP kernels (implemented in kernels.hip and blas.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "bodies.h"
#include "bodies_metric.h"
#include "constants.h"

namespace pmg {

// Workgroup arena of a kernel: in LDS when it fits the device limit, otherwise a slice of
// a global-memory buffer (then the grid is capped at `slots` workgroups that loop).
struct Arena {
  void *global = nullptr;  // device buffer, or nullptr when every kernel fits in LDS
  int slots = 0;           // workgroups the global buffer has room for
  size_t lds_max = 0;      // bytes of LDS a workgroup may use on this device
  int ncu = 256;           // compute units of the device
  int patch_lanes = 0;     // PMG_LANES_*: lanes per patch of the Cartesian smoother
};

// Patch launches with at most this many patches per CU use the 256-lane latency variant
// (unless the problem's configuration fixes the lane count).
constexpr int kWideLaunch = 4;

// FP32 launches of the 3D degree-4 and degree-5 default-solver kernels with at least this many
// patches per CU run half the per-degree lanes per patch (one wave at degree 4, two at degree
// 5; unless the configuration fixes the lane count): their FP32 arenas let 27 and 14 patches
// share a CU, which the per-degree count (two and four waves) would cap at 16 and 8 (32 waves
// per CU), and fewer lanes per patch leave fewer of them idle in the short contraction
// stages.  Smaller launches keep the per-degree count, which finishes each patch sooner; FP64
// patches (13 and 7 per CU by LDS whatever their lane count) measured the same or slower with
// fewer lanes and keep it.
constexpr int kHalfLaunch = 64;

// Bytes of LDS a workgroup may use on the current device (queried once per process).
inline size_t device_lds_limit() {
  static const size_t v = [] {
    int d = 0, l = 0;
    if (hipGetDevice(&d) != hipSuccess ||
        hipDeviceGetAttribute(&l, hipDeviceAttributeMaxSharedMemoryPerBlock, d) != hipSuccess)
      return (size_t)0;
    return (size_t)l;
  }();
  return v;
}

// Kernel launchers of one (dimension, precision); instantiated in kernels_<d>d_<prec>.hip.
template <int DIM, typename T>
struct Launchers {
  static size_t patch_bytes(int p, int hcode);
  static size_t apply_bytes(int p);
  static int smooth(int p, int hcode, const SmoothArgs<T> &a, const Arena &ar, hipStream_t s);
  static int local(int p, int hcode, const SmoothArgs<T> &a, int nb, const Arena &ar, hipStream_t s);
  // kind: 0 v = A u, 1 v = b - A u, 2 v = c M u
  static int apply(int p, int kind, const ApplyArgs<T> &a, const Arena &ar, hipStream_t s);
  static int restrict_(int p, const TransferArgs<T> &a, hipStream_t s);
  static int prolong(int p, const TransferArgs<T> &a, hipStream_t s);
  static int coarse(const CoarseArgs<T> &a, hipStream_t s);
};

// Launchers of the general (metric) path; instantiated in kernels_metric_*.hip for
// (3D, 2D) x (double/double, float/float) and 3D float/bfloat16.
template <int DIM, typename T, typename S>
struct MetricLaunchers {
  static size_t patch_bytes(int p);
  static size_t apply_bytes(int p);
  static int smooth(int p, const MetricSmoothArgs<T, S> &a, const Arena &ar, hipStream_t s);
  static int local(int p, const MetricSmoothArgs<T, S> &a, int nb, const Arena &ar, hipStream_t s);
  static int apply(int p, const MetricApplyArgs<T, S> &a, const Arena &ar, hipStream_t s);
  static int apply_init(int m, bool resid, const T *b, const T *u, T *out, hipStream_t s);
};

// Setup and coarse-solve kernels of the general path (setup.hip).
// cdiag[cell * (q+1)^d + node] = diagonal of the element matrix of degree q (metric G, FP64)
int launch_cell_diag(int dim, int q, long n_cells, const double *B, const double *Dn, const double *G, double *cdiag,
                     hipStream_t s);
// invD[patch * (2q-1)^d + e] = omega / (patch diagonal), stored as S
template <typename S>
int launch_patch_invdiag(int dim, int q, int n, double omega, const double *cdiag, S *invD, hipStream_t s);
int launch_set_identity(double *A, int m, hipStream_t s);
// z = Ainv r on interior nodes of an m0^d interior grid (total nodes per direction mt),
// z = r on boundary nodes; w is a work vector of m interior entries
template <typename T>
int launch_coarse_dense(int dim, int mi, int mt, const double *Ainv, const T *r, T *z, double *w, hipStream_t s);
template <typename S>
int launch_convert(const double *in, S *out, long n, hipStream_t s);

// Bytes of the per-workgroup arena of each kernel family (0 if not compiled in).
size_t patch_arena_bytes(int dim, int prec, int p, int hcode);
size_t apply_arena_bytes(int dim, int prec, int p);
size_t metric_patch_arena_bytes(int dim, int prec, int p);
size_t metric_apply_arena_bytes(int dim, int prec, int p);

template <typename T>
int launch_smooth_color(int dim, int p, int hcode, const SmoothArgs<T> &a, const Arena &ar, hipStream_t s);
template <typename T>
int launch_local_only(int dim, int p, int hcode, const SmoothArgs<T> &a, int n_blocks, const Arena &ar,
                      hipStream_t s);
template <typename T>
int launch_apply(int dim, int p, int kind, const ApplyArgs<T> &a, const Arena &ar, hipStream_t s);
template <typename T>
int launch_restrict(int dim, int p, const TransferArgs<T> &a, hipStream_t s);
template <typename T>
int launch_prolong_add(int dim, int p, const TransferArgs<T> &a, hipStream_t s);
template <typename T>
int launch_coarse(int dim, const CoarseArgs<T> &a, hipStream_t s);

// ---- vector kernels (blas.hip) ----
constexpr int kRedBlocks = 512;  // fixed grid of the deterministic reductions
enum Scal { S_RZ = 0, S_PQ, S_ALPHA, S_RR, S_ZRN, S_ZRO, S_BETA, S_BB, S_COUNT };

// partial[k*kRedBlocks + b] = block b's share of (x, y_k), k < ny (1 or 2)
int launch_dot_partial(const double *x, const double *y0, const double *y1, long n, double *partial,
                       hipStream_t s);
// final sums of the partials; mode selects the follow-up scalar update:
//  0: scal[i0] = (x,y0)                      1: scal[S_PQ] = (p,q), scal[S_ALPHA] = rz/pq
//  2: scal[S_ZRN], scal[S_ZRO]; beta = (zrn - zro)/rz; rz = zrn
int launch_dot_final(const double *partial, int ny, int mode, int i0, double *scal, hipStream_t s);
// x += alpha p; rn = ro - alpha q; partial (rn, rn)
int launch_fcg_xr(double *x, const double *ro, double *rn, const double *p, const double *q, const double *scal,
                  long n, double *partial, hipStream_t s);
// p = z + beta p
int launch_fcg_p(double *p, const double *z, const double *scal, long n, hipStream_t s);
int launch_copy(double *dst, const double *src, long n, hipStream_t s);
int launch_cast_d2f(const double *in, float *out, long n, hipStream_t s);
int launch_cast_f2d(const float *in, double *out, long n, hipStream_t s);
// z = 0 on interior nodes, z = r on boundary nodes of an m^dim node grid
template <typename T>
int launch_init_z(int dim, int m, T *z, const T *r, hipStream_t s);

}  // namespace pmg
