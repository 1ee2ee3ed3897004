// HIP kernels of the general path (distorted cells, variable coefficient): cellwise
// colored apply, metric patch smoother and local solve.  Instantiated once per
// (dimension, compute type, metric storage type) in kernels_metric_*.hip; only the
// paper's p-hierarchy is compiled for this path.
#pragma once

#include <hip/hip_runtime.h>

#include "bodies_metric.h"
#include "dispatch.h"
#include "hex_launch.h"
#include "launch.h"

namespace pmg {

namespace mdetail {

template <typename T>
__device__ inline T *lds_arena() {
  extern __shared__ __align__(16) unsigned char smem[];
  return reinterpret_cast<T *>(smem);
}

// ONE: the local solver is one half V-cycle (no post-smoothing, one Richardson step).
template <int DIM, typename T, typename S, int P, class H, bool ONE>
__global__ __launch_bounds__(metric_patch_threads(P, sizeof(T))) void k_msmooth(MetricSmoothArgs<T, S> a) {
  using B = MetricPatchBody<DIM, T, S, metric_patch_threads(P, sizeof(T)), P, H>;
  B::template smooth_patch<ONE>(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

template <int DIM, typename T, typename S, int P, class H>
__global__ __launch_bounds__(metric_patch_threads(P, sizeof(T))) void k_msmooth_g(MetricSmoothArgs<T, S> a, void *garena) {
  using B = MetricPatchBody<DIM, T, S, metric_patch_threads(P, sizeof(T)), P, H>;
  T *ar = reinterpret_cast<T *>(garena) + (size_t)blockIdx.x * B::size;
  for (int blk = blockIdx.x; blk < a.n_patch; blk += gridDim.x) {
    B::smooth_patch(threadIdx.x, blk, ar, a);
    __syncthreads();
  }
}

template <int DIM, typename T, typename S, int P, class H>
__global__ __launch_bounds__(metric_patch_threads(P, sizeof(T))) void k_mlocal(MetricSmoothArgs<T, S> a, int nb) {
  using B = MetricPatchBody<DIM, T, S, metric_patch_threads(P, sizeof(T)), P, H>;
  B::local_only(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

template <int DIM, typename T, typename S, int P, class H>
__global__ __launch_bounds__(metric_patch_threads(P, sizeof(T))) void k_mlocal_g(MetricSmoothArgs<T, S> a, int nb,
                                                                       void *garena) {
  using B = MetricPatchBody<DIM, T, S, metric_patch_threads(P, sizeof(T)), P, H>;
  T *ar = reinterpret_cast<T *>(garena) + (size_t)blockIdx.x * B::size;
  for (int blk = blockIdx.x; blk < nb; blk += gridDim.x) {
    B::local_only(threadIdx.x, blk, ar, a);
    __syncthreads();
  }
}

template <int DIM, typename T, typename S, int P>
__global__ __launch_bounds__(metric_apply_threads(P)) void k_mapply(MetricApplyArgs<T, S> a) {
  using B = MetricApplyBody<DIM, T, S, metric_apply_threads(P), P>;
  B::run(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

template <int DIM, typename T, typename S, int P>
__global__ __launch_bounds__(metric_apply_threads(P)) void k_mapply_g(MetricApplyArgs<T, S> a, void *garena) {
  using B = MetricApplyBody<DIM, T, S, metric_apply_threads(P), P>;
  T *ar = reinterpret_cast<T *>(garena) + (size_t)blockIdx.x * B::size;
  for (int blk = blockIdx.x; blk < a.n_cells; blk += gridDim.x) {
    B::run(threadIdx.x, blk, ar, a);
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_minit(int dim, int m, int resid, const T *b, const T *u, T *out, long n) {
  const long g = (long)blockIdx.x * 256 + threadIdx.x;
  if (g < n) metric_apply_init<T>(g, dim, m, resid != 0, b, u, out);
}

// general hex meshes: the same bodies through the stored maps
template <int DIM, typename T, int P, class H, bool ONE>
__global__ __launch_bounds__(metric_patch_threads(P, sizeof(T))) void k_hsmooth(MetricSmoothArgs<T, T> a) {
  using B = MetricPatchBody<DIM, T, T, metric_patch_threads(P, sizeof(T)), P, H>;
  B::template smooth_patch_stored<ONE>(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

template <int DIM, typename T, int P, class H>
__global__ __launch_bounds__(metric_patch_threads(P, sizeof(T))) void k_hsmooth_g(MetricSmoothArgs<T, T> a,
                                                                            void *garena) {
  using B = MetricPatchBody<DIM, T, T, metric_patch_threads(P, sizeof(T)), P, H>;
  T *ar = reinterpret_cast<T *>(garena) + (size_t)blockIdx.x * B::size;
  for (int blk = blockIdx.x; blk < a.n_patch; blk += gridDim.x) {
    B::smooth_patch_stored(threadIdx.x, blk, ar, a);
    __syncthreads();
  }
}

template <int DIM, typename T, int P>
__global__ __launch_bounds__(metric_apply_threads(P)) void k_happly(MetricApplyArgs<T, T> a) {
  using B = MetricApplyBody<DIM, T, T, metric_apply_threads(P), P>;
  B::template run<true>(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

template <int DIM, typename T, int P>
__global__ __launch_bounds__(metric_apply_threads(P)) void k_happly_g(MetricApplyArgs<T, T> a, void *garena) {
  using B = MetricApplyBody<DIM, T, T, metric_apply_threads(P), P>;
  T *ar = reinterpret_cast<T *>(garena) + (size_t)blockIdx.x * B::size;
  for (int blk = blockIdx.x; blk < a.n_cells; blk += gridDim.x) {
    B::template run<true>(threadIdx.x, blk, ar, a);
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_hinit(int resid, const unsigned char *bnd, const T *b, const T *u, T *out,
                                               long n) {
  const long g = (long)blockIdx.x * 256 + threadIdx.x;
  if (g < n) hex_apply_init<T>(g, resid != 0, bnd, b, u, out);
}

template <typename KL, typename KG, typename... Args>
int launch_arena(KL klds, KG kglob, int nblk, int threads, size_t bytes, const Arena &ar, hipStream_t s,
                 Args... args) {
  if (nblk <= 0) return 0;
  if (bytes > ar.lds_max) {
    if (!ar.global || ar.slots <= 0) return -3;
    const int grid = nblk < ar.slots ? nblk : ar.slots;
    hipLaunchKernelGGL(kglob, dim3(grid), dim3(threads), 0, s, args..., ar.global);
  } else {
    if (bytes > 65536) {
      static thread_local const void *last = nullptr;
      if (last != (const void *)klds) {
        if (hipFuncSetAttribute((const void *)klds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ar.lds_max) !=
            hipSuccess)
          return -4;
        last = (const void *)klds;
      }
    }
    hipLaunchKernelGGL(klds, dim3(nblk), dim3(threads), bytes, s, args...);
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <int DIM, typename T, typename S>
struct SmoothF {
  template <int P, class H>
  struct F {
    static int run(const MetricSmoothArgs<T, S> &a, const Arena &ar, hipStream_t s) {
      using B = MetricPatchBody<DIM, T, S, metric_patch_threads(P, sizeof(T)), P, H>;
      const size_t bytes = B::arena(a.n_iter) * sizeof(T);
      if (a.full == 0 && a.n_iter == 1)
        return launch_arena(k_msmooth<DIM, T, S, P, H, true>, k_msmooth_g<DIM, T, S, P, H>, a.n_patch,
                            metric_patch_threads(P, sizeof(T)), bytes, ar, s, a);
      return launch_arena(k_msmooth<DIM, T, S, P, H, false>, k_msmooth_g<DIM, T, S, P, H>, a.n_patch,
                          metric_patch_threads(P, sizeof(T)), bytes, ar, s, a);
    }
  };
};

template <int DIM, typename T, typename S>
struct LocalF {
  template <int P, class H>
  struct F {
    static int run(const MetricSmoothArgs<T, S> &a, int nb, const Arena &ar, hipStream_t s) {
      using B = MetricPatchBody<DIM, T, S, metric_patch_threads(P, sizeof(T)), P, H>;
      return launch_arena(k_mlocal<DIM, T, S, P, H>, k_mlocal_g<DIM, T, S, P, H>, nb, metric_patch_threads(P, sizeof(T)),
                          B::arena(a.n_iter) * sizeof(T), ar, s, a, nb);
    }
  };
};

template <int DIM, typename T, typename S>
struct PatchBytesF {
  template <int P, class H>
  struct F {
    static int run(size_t *out) {
      *out = MetricPatchBody<DIM, T, S, metric_patch_threads(P, sizeof(T)), P, H>::size * sizeof(T);
      return 0;
    }
  };
};

template <int DIM, typename T, typename S>
struct ApplyF {
  template <int P>
  struct F {
    static int run(const MetricApplyArgs<T, S> &a, const Arena &ar, hipStream_t s) {
      using B = MetricApplyBody<DIM, T, S, metric_apply_threads(P), P>;
      return launch_arena(k_mapply<DIM, T, S, P>, k_mapply_g<DIM, T, S, P>, a.n_cells, metric_apply_threads(P),
                          B::size * sizeof(T), ar, s, a);
    }
  };
};

template <int DIM, typename T, typename S>
struct ApplyBytesF {
  template <int P>
  struct F {
    static int run(size_t *out) {
      *out = MetricApplyBody<DIM, T, S, metric_apply_threads(P), P>::size * sizeof(T);
      return 0;
    }
  };
};

template <int DIM, typename T>
struct HSmoothF {
  template <int P, class H>
  struct F {
    static int run(const MetricSmoothArgs<T, T> &a, const Arena &ar, hipStream_t s) {
      using B = MetricPatchBody<DIM, T, T, metric_patch_threads(P, sizeof(T)), P, H>;
      const size_t bytes = B::arena(a.n_iter) * sizeof(T);
      if (a.full == 0 && a.n_iter == 1)
        return launch_arena(k_hsmooth<DIM, T, P, H, true>, k_hsmooth_g<DIM, T, P, H>, a.n_patch,
                            metric_patch_threads(P, sizeof(T)), bytes, ar, s, a);
      return launch_arena(k_hsmooth<DIM, T, P, H, false>, k_hsmooth_g<DIM, T, P, H>, a.n_patch,
                          metric_patch_threads(P, sizeof(T)), bytes, ar, s, a);
    }
  };
};

template <int DIM, typename T>
struct HApplyF {
  template <int P>
  struct F {
    static int run(const MetricApplyArgs<T, T> &a, const Arena &ar, hipStream_t s) {
      using B = MetricApplyBody<DIM, T, T, metric_apply_threads(P), P>;
      return launch_arena(k_happly<DIM, T, P>, k_happly_g<DIM, T, P>, a.n_cells, metric_apply_threads(P),
                          B::size * sizeof(T), ar, s, a);
    }
  };
};

}  // namespace mdetail

template <int DIM, typename T>
size_t HexLaunchers<DIM, T>::patch_bytes(int p) {
  return MetricLaunchers<DIM, T, T>::patch_bytes(p);
}

template <int DIM, typename T>
size_t HexLaunchers<DIM, T>::apply_bytes(int p) {
  return MetricLaunchers<DIM, T, T>::apply_bytes(p);
}

template <int DIM, typename T>
int HexLaunchers<DIM, T>::smooth(int p, const MetricSmoothArgs<T, T> &a, const Arena &ar, hipStream_t s) {
  return dispatch_hierarchy<mdetail::HSmoothF<DIM, T>::template F>(p, 0, a, ar, s);
}

template <int DIM, typename T>
int HexLaunchers<DIM, T>::apply(int p, const MetricApplyArgs<T, T> &a, const Arena &ar, hipStream_t s) {
  return dispatch_degree<mdetail::HApplyF<DIM, T>::template F>(p, a, ar, s);
}

template <int DIM, typename T>
int HexLaunchers<DIM, T>::apply_init(long n, bool resid, const unsigned char *bnd, const T *b, const T *u, T *out,
                                     hipStream_t s) {
  hipLaunchKernelGGL((mdetail::k_hinit<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (int)resid, bnd, b, u,
                     out, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <int DIM, typename T, typename S>
size_t MetricLaunchers<DIM, T, S>::patch_bytes(int p) {
  size_t out = 0;
  return dispatch_hierarchy<mdetail::PatchBytesF<DIM, T, S>::template F>(p, 0, &out) == 0 ? out : 0;
}

template <int DIM, typename T, typename S>
size_t MetricLaunchers<DIM, T, S>::apply_bytes(int p) {
  size_t out = 0;
  return dispatch_degree<mdetail::ApplyBytesF<DIM, T, S>::template F>(p, &out) == 0 ? out : 0;
}

template <int DIM, typename T, typename S>
int MetricLaunchers<DIM, T, S>::smooth(int p, const MetricSmoothArgs<T, S> &a, const Arena &ar, hipStream_t s) {
  return dispatch_hierarchy<mdetail::SmoothF<DIM, T, S>::template F>(p, 0, a, ar, s);
}

template <int DIM, typename T, typename S>
int MetricLaunchers<DIM, T, S>::local(int p, const MetricSmoothArgs<T, S> &a, int nb, const Arena &ar,
                                      hipStream_t s) {
  return dispatch_hierarchy<mdetail::LocalF<DIM, T, S>::template F>(p, 0, a, nb, ar, s);
}

template <int DIM, typename T, typename S>
int MetricLaunchers<DIM, T, S>::apply(int p, const MetricApplyArgs<T, S> &a, const Arena &ar, hipStream_t s) {
  return dispatch_degree<mdetail::ApplyF<DIM, T, S>::template F>(p, a, ar, s);
}

template <int DIM, typename T, typename S>
int MetricLaunchers<DIM, T, S>::apply_init(int m, bool resid, const T *b, const T *u, T *out, hipStream_t s) {
  const long n = DIM == 3 ? (long)m * m * m : (long)m * m;
  hipLaunchKernelGGL((mdetail::k_minit<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, DIM, m, (int)resid,
                     b, u, out, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace pmg
