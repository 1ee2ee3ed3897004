// HIP kernels of the patch smoother, the operator apply, the h-transfers and the coarse
// solve, for gfx950.  The bodies live in bodies.h; this header owns launch shapes and is
// instantiated once per (dimension, precision) in kernels_<dim>_<prec>.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "launch.h"

namespace pmg {

namespace detail {

// Each workgroup kernel comes in two variants: the arena in LDS (dynamic shared memory,
// so every arena access compiles to ds_read/ds_write), or, when the arena exceeds the
// device's LDS limit, a slice of a global buffer with a grid-stride loop.
template <typename T>
__device__ inline T *lds_arena() {
  extern __shared__ __align__(16) unsigned char smem[];
  return reinterpret_cast<T *>(smem);
}

// ---- patch smoother: one workgroup per patch of one color ----
// ONE: the local solver is one half V-cycle (no post-smoothing, one Richardson step).
template <int DIM, typename T, int P, class H, bool ONE>
__global__ __launch_bounds__(patch_threads(P, DIM, sizeof(T))) void k_smooth(SmoothArgs<T> a) {
  using B = PatchBody<DIM, T, patch_threads(P, DIM, sizeof(T)), P, H>;
  B::template smooth_patch<ONE>(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

// Latency variant for small launches (few patches per CU, as on coarse h-levels): 256
// lanes per patch, so that the short contraction stages split their outputs over four
// waves and each patch finishes sooner.
template <int DIM, typename T, int P, class H, bool ONE>
__global__ __launch_bounds__(256) void k_smooth_w(SmoothArgs<T> a) {
  using B = PatchBody<DIM, T, 256, P, H>;
  B::template smooth_patch<ONE>(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

// Half the per-degree lanes per patch (NT: one wave at 3D degree 4, two at degree 5), for the
// largest launches of the default local solver.
template <int DIM, typename T, int P, class H, int NT>
__global__ __launch_bounds__(NT) void k_smooth_h(SmoothArgs<T> a) {
  using B = PatchBody<DIM, T, NT, P, H>;
  B::template smooth_patch<true>(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

template <int DIM, typename T, int P, class H>
__global__ __launch_bounds__(patch_threads(P, DIM, sizeof(T))) void k_smooth_g(SmoothArgs<T> a, void *garena) {
  using B = PatchBody<DIM, T, patch_threads(P, DIM, sizeof(T)), P, H>;
  T *ar = reinterpret_cast<T *>(garena) + (size_t)blockIdx.x * B::size;
  for (int blk = blockIdx.x; blk < a.n_patch; blk += gridDim.x) {
    B::smooth_patch(threadIdx.x, blk, ar, a);
    __syncthreads();
  }
}

template <int DIM, typename T, int P, class H>
__global__ __launch_bounds__(patch_threads(P, DIM, sizeof(T))) void k_local(SmoothArgs<T> a, int n_blocks) {
  using B = PatchBody<DIM, T, patch_threads(P, DIM, sizeof(T)), P, H>;
  B::local_only(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

template <int DIM, typename T, int P, class H>
__global__ __launch_bounds__(patch_threads(P, DIM, sizeof(T))) void k_local_g(SmoothArgs<T> a, int n_blocks, void *garena) {
  using B = PatchBody<DIM, T, patch_threads(P, DIM, sizeof(T)), P, H>;
  T *ar = reinterpret_cast<T *>(garena) + (size_t)blockIdx.x * B::size;
  for (int blk = blockIdx.x; blk < n_blocks; blk += gridDim.x) {
    B::local_only(threadIdx.x, blk, ar, a);
    __syncthreads();
  }
}

// ---- operator apply: one workgroup per tile ----
template <int DIM, typename T, int P, bool RESID, bool MASS>
__global__ __launch_bounds__(apply_threads(P)) void k_apply(ApplyArgs<T> a) {
  using B = ApplyBody<DIM, T, apply_threads(P), P, tile_cells(P), RESID, MASS>;
  B::run(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

template <int DIM, typename T, int P, bool RESID, bool MASS>
__global__ __launch_bounds__(apply_threads(P)) void k_apply_g(ApplyArgs<T> a, void *garena) {
  using B = ApplyBody<DIM, T, apply_threads(P), P, tile_cells(P), RESID, MASS>;
  T *ar = reinterpret_cast<T *>(garena) + (size_t)blockIdx.x * B::size;
  for (int blk = blockIdx.x; blk < a.n_tiles; blk += gridDim.x) {
    B::run(threadIdx.x, blk, ar, a);
    __syncthreads();
  }
}

// ---- operator apply marching in z: one workgroup per xy tile and z segment (3D) ----
template <typename T, int P, bool RESID = false, bool MASS = false>
using March = MarchBody<T, march_threads(P), P, march_tile(P), march_tile_y(P), march_group(P),
                        P * (tile_cells(P) + 1) + 1, RESID, MASS>;

template <typename T, int P, bool RESID, bool MASS>
__global__ __launch_bounds__(march_threads(P)) void k_march(ApplyArgs<T> a) {
  using B = March<T, P, RESID, MASS>;
  B::run(threadIdx.x, blockIdx.x, lds_arena<T>(), a);
}

// ---- h-transfer: one 1D pass, one thread per output entry ----
template <typename T, int P, bool RESTRICT, bool ADD>
__global__ __launch_bounds__(256) void k_transfer(PassArgs<T> a, long total) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < total) TransferPass<T, P, RESTRICT, ADD>::node(g, a);
}

template <int DIM, typename T>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse(CoarseArgs<T> a, int lds_elems) {
  CoarseBody<DIM, T, kCoarseThreads>::run(threadIdx.x, a, lds_arena<double>(), lds_elems);
}

// Launch the LDS variant with `bytes` of dynamic shared memory, or the global-arena
// variant (grid capped at the arena's slots) when the arena does not fit in LDS.
template <typename KL, typename KG, typename... Args>
int launch_arena(KL klds, KG kglob, int nblk, int threads, size_t bytes, const Arena &ar, hipStream_t s,
                 Args... args) {
  if (nblk <= 0) return 0;
  if (bytes > ar.lds_max) {
    if (!ar.global || ar.slots <= 0) return -3;
    const int grid = nblk < ar.slots ? nblk : ar.slots;
    hipLaunchKernelGGL(kglob, dim3(grid), dim3(threads), 0, s, args..., ar.global);
  } else {
    if (bytes > 65536) {  // raise the kernel's limit once, to the device maximum
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

template <typename T>
struct SmoothL {
  template <int DIM>
  struct D {
    template <int P, class H>
    struct F {
      static int run(const SmoothArgs<T> &a, const Arena &ar, hipStream_t s) {
        using B = PatchBody<DIM, T, patch_threads(P, DIM, sizeof(T)), P, H>;
        const bool one = a.full == 0 && a.n_iter == 1 && a.direct == 0 && a.reinf == 0;
        const size_t bytes = (one ? B::arena_one() : B::arena(a.n_iter)) * sizeof(T);
        // patch_lanes: 0 by launch size, 1 always the per-degree count, 2 always 256, 3 half the
        // per-degree count where the degree has that variant (else the per-degree count)
        const bool wide = ar.patch_lanes == 2 || (ar.patch_lanes == 0 && a.n_patch <= kWideLaunch * ar.ncu);
        constexpr int PT = patch_threads(P, DIM, sizeof(T));
        if constexpr (DIM == 3 && (P == 4 || P == 5) && PT >= 128) {
          const bool half =
              ar.patch_lanes == 3 || (ar.patch_lanes == 0 && sizeof(T) == 4 && a.n_patch >= kHalfLaunch * ar.ncu);
          if (one && half && bytes <= ar.lds_max)
            return launch_arena(k_smooth_h<DIM, T, P, H, PT / 2>, k_smooth_g<DIM, T, P, H>, a.n_patch, PT / 2, bytes,
                                ar, s, a);
        }
        if constexpr (patch_threads(P, DIM, sizeof(T)) < 256)
          if (wide && bytes <= ar.lds_max)
            return one ? launch_arena(k_smooth_w<DIM, T, P, H, true>, k_smooth_g<DIM, T, P, H>, a.n_patch, 256,
                                      bytes, ar, s, a)
                       : launch_arena(k_smooth_w<DIM, T, P, H, false>, k_smooth_g<DIM, T, P, H>, a.n_patch, 256,
                                      bytes, ar, s, a);
        return one ? launch_arena(k_smooth<DIM, T, P, H, true>, k_smooth_g<DIM, T, P, H>, a.n_patch,
                                  patch_threads(P, DIM, sizeof(T)), bytes, ar, s, a)
                   : launch_arena(k_smooth<DIM, T, P, H, false>, k_smooth_g<DIM, T, P, H>, a.n_patch,
                                  patch_threads(P, DIM, sizeof(T)), bytes, ar, s, a);
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
        using B = PatchBody<DIM, T, patch_threads(P, DIM, sizeof(T)), P, H>;
        return launch_arena(k_local<DIM, T, P, H>, k_local_g<DIM, T, P, H>, nb, patch_threads(P, DIM, sizeof(T)),
                            B::arena(a.n_iter) * sizeof(T), ar, s, a, nb);
      }
    };
  };
};

template <typename T, int DIM>
struct SizeL {
  template <int P, class H>
  struct F {
    static int run(size_t *out) {
      *out = PatchBody<DIM, T, patch_threads(P, DIM, sizeof(T)), P, H>::size * sizeof(T);
      return 0;
    }
  };
};

template <typename T, int DIM>
struct ApplySizeL {
  template <int P>
  struct F {
    static int run(size_t *out) {
      if constexpr (DIM == 3 && march_tile(P) > 0)
        *out = March<T, P>::size * sizeof(T);
      else
        *out = ApplyBody<DIM, T, apply_threads(P), P, tile_cells(P), false>::size * sizeof(T);
      return 0;
    }
  };
};

// KIND: 0 v = A u, 1 v = b - A u, 2 v = c M u (the mass matrix)
template <typename T, int DIM, int KIND>
struct ApplyL {
  static constexpr bool RESID = KIND == 1, MASS = KIND == 2;
  template <int P>
  struct F {
    static int run(const ApplyArgs<T> &a, const Arena &ar, hipStream_t s) {
      if constexpr (DIM == 3 && march_tile(P) > 0) if (march_fits<T>(P, (long)P * a.n + 1)) {
        constexpr size_t bytes = March<T, P>::size * sizeof(T);
        if (bytes > ar.lds_max) return -3;
        if (bytes > 65536) {  // raise the kernel's limit once, to the device maximum
          static thread_local bool raised = false;
          if (!raised) {
            if (hipFuncSetAttribute((const void *)k_march<T, P, RESID, MASS>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)ar.lds_max) != hipSuccess)
              return -4;
            raised = true;
          }
        }
        ApplyArgs<T> b = a;
        int nseg;
        march_geometry(a.n, march_tile(P), march_tile_y(P), kMarchBlocks, b.mt, b.mty, nseg, b.zc);
        b.n_tiles = b.mt * b.mty * nseg;
        hipLaunchKernelGGL((k_march<T, P, RESID, MASS>), dim3(b.n_tiles), dim3(march_threads(P)), bytes, s, b);
        return hipGetLastError() == hipSuccess ? 0 : -4;
      }
      using B = ApplyBody<DIM, T, apply_threads(P), P, tile_cells(P), RESID, MASS>;
      return launch_arena(k_apply<DIM, T, P, RESID, MASS>, k_apply_g<DIM, T, P, RESID, MASS>, a.n_tiles,
                          apply_threads(P), B::size * sizeof(T), ar, s, a);
    }
  };
};

template <typename T, int DIM, bool RESTRICT>
struct TransferL {
  template <int P>
  struct F {
    static int run(const TransferArgs<T> &a, hipStream_t s) {
      PassArgs<T> pa[3];
      const int np = transfer_passes<T>(DIM, P, RESTRICT, a, pa);
      for (int k = 0; k < np; ++k) {
        const long total = (long)pa[k].oe[0] * pa[k].oe[1] * pa[k].oe[2];
        const int grid = (int)((total + 255) / 256);
        if (RESTRICT)
          hipLaunchKernelGGL((k_transfer<T, P, true, false>), dim3(grid), dim3(256), 0, s, pa[k], total);
        else if (k == np - 1)
          hipLaunchKernelGGL((k_transfer<T, P, false, true>), dim3(grid), dim3(256), 0, s, pa[k], total);
        else
          hipLaunchKernelGGL((k_transfer<T, P, false, false>), dim3(grid), dim3(256), 0, s, pa[k], total);
        if (hipGetLastError() != hipSuccess) return -4;
      }
      return 0;
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
int Launchers<DIM, T>::apply(int p, int kind, const ApplyArgs<T> &a, const Arena &ar, hipStream_t s) {
  switch (kind) {
    case 0: return dispatch_degree<detail::ApplyL<T, DIM, 0>::template F>(p, a, ar, s);
    case 1: return dispatch_degree<detail::ApplyL<T, DIM, 1>::template F>(p, a, ar, s);
    case 2: return dispatch_degree<detail::ApplyL<T, DIM, 2>::template F>(p, a, ar, s);
    default: return -1;
  }
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
  // the two work vectors of the fast diagonalization in workgroup memory when they fit
  const size_t tot = DIM == 3 ? (size_t)a.m * a.m * a.m : (size_t)a.m * a.m;
  size_t bytes = 2 * tot * sizeof(double);
  if (bytes > device_lds_limit()) bytes = 0;
  if (bytes > 65536) {
    static thread_local bool raised = false;
    if (!raised) {
      if (hipFuncSetAttribute((const void *)detail::k_coarse<DIM, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)device_lds_limit()) != hipSuccess)
        return -4;
      raised = true;
    }
  }
  hipLaunchKernelGGL((detail::k_coarse<DIM, T>), dim3(1), dim3(kCoarseThreads), bytes, s, a,
                     (int)(bytes / sizeof(double)));
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace pmg
