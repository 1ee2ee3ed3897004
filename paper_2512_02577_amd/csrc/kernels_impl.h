// HIP kernels of the patch smoother, the operator apply, the h-transfers and the coarse
// solve, for gfx950.  The bodies live in bodies.h; this header owns launch shapes and is
// instantiated once per (dimension, precision) in kernels_<dim>_<prec>.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "launch.h"

namespace pmg {

namespace detail {

template <typename T>
__device__ inline T *arena_ptr(void *global, size_t elems) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (global) return reinterpret_cast<T *>(global) + (size_t)blockIdx.x * elems;
  return reinterpret_cast<T *>(smem);
}

// ---- patch smoother: one workgroup per patch of one color ----
template <int DIM, typename T, int P, class H>
__global__ __launch_bounds__(patch_threads(P)) void k_smooth(SmoothArgs<T> a, void *garena) {
  using B = PatchBody<DIM, T, patch_threads(P), P, H>;
  T *lds = arena_ptr<T>(garena, B::size);
  for (int blk = blockIdx.x; blk < a.n_patch; blk += gridDim.x) {
    B::smooth_patch(threadIdx.x, blk, lds, a);
    __syncthreads();
  }
}

template <int DIM, typename T, int P, class H>
__global__ __launch_bounds__(patch_threads(P)) void k_local(SmoothArgs<T> a, int n_blocks, void *garena) {
  using B = PatchBody<DIM, T, patch_threads(P), P, H>;
  T *lds = arena_ptr<T>(garena, B::size);
  for (int blk = blockIdx.x; blk < n_blocks; blk += gridDim.x) {
    B::local_only(threadIdx.x, blk, lds, a);
    __syncthreads();
  }
}

// ---- operator apply: one workgroup per tile ----
template <int DIM, typename T, int P, bool RESID>
__global__ __launch_bounds__(apply_threads(P)) void k_apply(ApplyArgs<T> a, void *garena) {
  using B = ApplyBody<DIM, T, apply_threads(P), P, tile_cells(P), RESID>;
  T *lds = arena_ptr<T>(garena, B::size);
  for (int blk = blockIdx.x; blk < a.n_tiles; blk += gridDim.x) {
    B::run(threadIdx.x, blk, lds, a);
    __syncthreads();
  }
}

template <int DIM, typename T, int P>
__global__ __launch_bounds__(256) void k_restrict(TransferArgs<T> a, long total) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < total) TransferBody<DIM, T, P>::restrict_node(g, a);
}

template <int DIM, typename T, int P>
__global__ __launch_bounds__(256) void k_prolong(TransferArgs<T> a, long total) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < total) TransferBody<DIM, T, P>::prolong_node(g, a);
}

template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_coarse(CoarseArgs<T> a) {
  CoarseBody<DIM, T, 256>::run(threadIdx.x, a);
}

// Launch with `bytes` of dynamic LDS (or the global arena when it does not fit).
template <typename K, typename... Args>
int launch_arena(K kernel, int nblk, int threads, size_t bytes, const Arena &ar, hipStream_t s, Args... args) {
  if (nblk <= 0) return 0;
  void *g = nullptr;
  size_t shmem = bytes;
  int grid = nblk;
  if (bytes > ar.lds_max) {
    if (!ar.global || ar.slots <= 0) return -3;
    g = ar.global;
    shmem = 0;
    grid = nblk < ar.slots ? nblk : ar.slots;
  } else if (bytes > 65536) {
    static thread_local const void *last = nullptr;
    if (last != (const void *)kernel) {
      if (hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
          hipSuccess)
        return -4;
      last = (const void *)kernel;
    }
  }
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), shmem, s, args..., g);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <typename T>
struct SmoothL {
  template <int DIM>
  struct D {
    template <int P, class H>
    struct F {
      static int run(const SmoothArgs<T> &a, const Arena &ar, hipStream_t s) {
        using B = PatchBody<DIM, T, patch_threads(P), P, H>;
        return launch_arena(k_smooth<DIM, T, P, H>, a.n_patch, patch_threads(P), B::size * sizeof(T), ar, s, a);
      }
    };
  };
};

template <typename T>
struct LocalL {
  template <int DIM>
  struct D {
    template <int P, class H>
    struct F {
      static int run(const SmoothArgs<T> &a, int nb, const Arena &ar, hipStream_t s) {
        using B = PatchBody<DIM, T, patch_threads(P), P, H>;
        return launch_arena(k_local<DIM, T, P, H>, nb, patch_threads(P), B::size * sizeof(T), ar, s, a, nb);
      }
    };
  };
};

template <typename T, int DIM>
struct SizeL {
  template <int P, class H>
  struct F {
    static int run(size_t *out) {
      *out = PatchBody<DIM, T, patch_threads(P), P, H>::size * sizeof(T);
      return 0;
    }
  };
};

template <typename T, int DIM>
struct ApplySizeL {
  template <int P>
  struct F {
    static int run(size_t *out) {
      *out = ApplyBody<DIM, T, apply_threads(P), P, tile_cells(P), false>::size * sizeof(T);
      return 0;
    }
  };
};

template <typename T, int DIM, bool RESID>
struct ApplyL {
  template <int P>
  struct F {
    static int run(const ApplyArgs<T> &a, const Arena &ar, hipStream_t s) {
      using B = ApplyBody<DIM, T, apply_threads(P), P, tile_cells(P), RESID>;
      return launch_arena(k_apply<DIM, T, P, RESID>, a.n_tiles, apply_threads(P), B::size * sizeof(T), ar, s, a);
    }
  };
};

template <typename T, int DIM, bool RESTRICT>
struct TransferL {
  template <int P>
  struct F {
    static int run(const TransferArgs<T> &a, hipStream_t s) {
      long m = RESTRICT ? (long)P * a.nc + 1 : 2L * P * a.nc + 1;
      long total = DIM == 3 ? m * m * m : m * m;
      int grid = (int)((total + 255) / 256);
      if (RESTRICT)
        hipLaunchKernelGGL((k_restrict<DIM, T, P>), dim3(grid), dim3(256), 0, s, a, total);
      else
        hipLaunchKernelGGL((k_prolong<DIM, T, P>), dim3(grid), dim3(256), 0, s, a, total);
      return hipGetLastError() == hipSuccess ? 0 : -4;
    }
  };
};

}  // namespace detail

template <int DIM, typename T>
size_t Launchers<DIM, T>::patch_bytes(int p, int hcode) {
  size_t out = 0;
  return dispatch_hierarchy<detail::SizeL<T, DIM>::template F>(p, hcode, &out) == 0 ? out : 0;
}
template <int DIM, typename T>
size_t Launchers<DIM, T>::apply_bytes(int p) {
  size_t out = 0;
  return dispatch_degree<detail::ApplySizeL<T, DIM>::template F>(p, &out) == 0 ? out : 0;
}
template <int DIM, typename T>
int Launchers<DIM, T>::smooth(int p, int hcode, const SmoothArgs<T> &a, const Arena &ar, hipStream_t s) {
  return dispatch_hierarchy<detail::SmoothL<T>::template D<DIM>::template F>(p, hcode, a, ar, s);
}
template <int DIM, typename T>
int Launchers<DIM, T>::local(int p, int hcode, const SmoothArgs<T> &a, int nb, const Arena &ar, hipStream_t s) {
  return dispatch_hierarchy<detail::LocalL<T>::template D<DIM>::template F>(p, hcode, a, nb, ar, s);
}
template <int DIM, typename T>
int Launchers<DIM, T>::apply(int p, bool resid, const ApplyArgs<T> &a, const Arena &ar, hipStream_t s) {
  return resid ? dispatch_degree<detail::ApplyL<T, DIM, true>::template F>(p, a, ar, s)
               : dispatch_degree<detail::ApplyL<T, DIM, false>::template F>(p, a, ar, s);
}
template <int DIM, typename T>
int Launchers<DIM, T>::restrict_(int p, const TransferArgs<T> &a, hipStream_t s) {
  return dispatch_degree<detail::TransferL<T, DIM, true>::template F>(p, a, s);
}
template <int DIM, typename T>
int Launchers<DIM, T>::prolong(int p, const TransferArgs<T> &a, hipStream_t s) {
  return dispatch_degree<detail::TransferL<T, DIM, false>::template F>(p, a, s);
}
template <int DIM, typename T>
int Launchers<DIM, T>::coarse(const CoarseArgs<T> &a, hipStream_t s) {
  hipLaunchKernelGGL((detail::k_coarse<DIM, T>), dim3(1), dim3(256), 0, s, a);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace pmg
