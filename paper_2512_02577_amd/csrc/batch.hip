// Batched stage kernels: persistent grids that walk the concatenated work items of all
// problems of one V-cycle stage, and the FP64 vector kernels of the batched outer CG.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "dispatch.h"
#include "launch.h"

namespace pmg {

namespace {

template <typename T>
__device__ inline T *lds_arena() {
  extern __shared__ __align__(16) unsigned char smem[];
  return reinterpret_cast<T *>(smem);
}

// Segment of work item `item` (segments sorted by start, at most kBatchMax of them).
template <typename Stage>
__device__ inline int seg_of(const cptr<Stage> &st, int nseg, long item) {
  int s = 0;
  while (s + 1 < nseg && st->seg[s + 1].start <= item) ++s;
  return s;
}

// The bodies read the arguments of a work item through a reference to its stage-table entry
// in the constant address space, field by field as they need them (scalar loads, as for kernel
// arguments); a local copy of the whole struct would hold every field in registers throughout
// the body.
template <typename A>
__device__ inline const A &table_ref(const PMG_CONST_AS A &x) {
  return *(const A *)&x;
}

// The lane index as a value the compiler cannot see through, taken anew in every iteration of
// a persistent loop: otherwise every index computation of the body that depends on the lane
// alone is hoisted out of the loop and held in registers across the whole body (more than
// twice the registers of the single-launch kernel, and lower occupancy).
template <int NT>
__device__ inline int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  __builtin_assume(t >= 0 && t < NT);  // the range the loops of the body rely on
  return t;
}

// One kernel per degree: the patch body of the single-problem kernel (same threads per
// workgroup, same registers) inside a loop over the work items of every segment.  ONE: every
// segment of the stage has the default local solver (one half V-cycle, one Richardson step),
// so the body compiled for it alone runs, with its smaller arena.
template <typename T, int P, bool ONE>
__global__ __launch_bounds__(patch_threads(P, 3, sizeof(T))) void k_bsmooth(const BSmoothStage<T> *st_) {
  using B = PatchBody<3, T, patch_threads(P, 3, sizeof(T)), P, typename PaperH<P>::type>;
  const cptr<BSmoothStage<T>> st = as_const(st_);
  T *lds = lds_arena<T>();
  const int nseg = st->nseg, total = st->total;
  for (int blk = blockIdx.x; blk < total; blk += gridDim.x) {
    const int s = seg_of(st, nseg, blk);
    if (!as_const(st->active)[st->seg[s].prob]) continue;
    const int local = blk - st->seg[s].start;
    if (local >= st->seg[s].a.n_patch) continue;  // padding of the segment to a multiple of 8
    B::template smooth_patch<ONE>(opaque_tid<patch_threads(P, 3, sizeof(T))>(), local, lds, table_ref(st->seg[s].a));
    __syncthreads();
  }
}

template <typename T, int P, bool RESID>
using BMarch = MarchBody<T, march_threads(P), P, march_tile(P), march_tile_y(P), march_group(P),
                         P * (tile_cells(P) + 1) + 1, RESID, false>;

// The marching apply of each segment's problem (apply option 0).
template <typename T, int P, bool RESID>
__global__ __launch_bounds__(march_threads(P)) void k_bmarch(const BApplyStage<T> *st_) {
  using B = BMarch<T, P, RESID>;
  const cptr<BApplyStage<T>> st = as_const(st_);
  T *lds = lds_arena<T>();
  const int nseg = st->nseg, total = st->total;
  for (int blk = blockIdx.x; blk < total; blk += gridDim.x) {
    const int s = seg_of(st, nseg, blk);
    if (!as_const(st->active)[st->seg[s].prob]) continue;
    const int local = blk - st->seg[s].start;
    if (local >= st->seg[s].a.n_tiles) continue;  // padding of the segment to a multiple of 8
    B::run(opaque_tid<march_threads(P)>(), local, lds, table_ref(st->seg[s].a));
    __syncthreads();
  }
}

// The owned-node tile apply (apply option 1).
template <typename T, int P, int OPT, bool RESID>
__global__ __launch_bounds__(apply_threads(P)) void k_bapply(const BApplyStage<T> *st_) {
  using B = ApplyBody<3, T, apply_threads(P), P, batch_tile(P, OPT), RESID>;
  const cptr<BApplyStage<T>> st = as_const(st_);
  T *lds = lds_arena<T>();
  const int nseg = st->nseg, total = st->total;
  for (int blk = blockIdx.x; blk < total; blk += gridDim.x) {
    const int s = seg_of(st, nseg, blk);
    if (!as_const(st->active)[st->seg[s].prob]) continue;
    const int local = blk - st->seg[s].start;
    if (local >= st->seg[s].a.n_tiles) continue;  // padding of the segment to a multiple of 8
    B::run(opaque_tid<apply_threads(P)>(), local, lds, table_ref(st->seg[s].a));
    __syncthreads();
  }
}

template <typename T, int P>
__device__ inline void pass_item(int mode, long g, const PassArgs<T> &pa) {
  if (mode == 0)
    TransferPass<T, P, true, false>::node(g, pa);
  else if (mode == 1)
    TransferPass<T, P, false, false>::node(g, pa);
  else
    TransferPass<T, P, false, true>::node(g, pa);
}

template <typename T>
__global__ __launch_bounds__(kBatchThreads) void k_bpass(const BPassStage<T> *st_) {
  const cptr<BPassStage<T>> st = as_const(st_);
  const int nseg = st->nseg;
  const long tt = st->total_threads;
  for (long g0 = (long)blockIdx.x * kBatchThreads; g0 < tt; g0 += (long)gridDim.x * kBatchThreads) {
    // segments start at multiples of the workgroup size: the segment is uniform per block
    const int s = seg_of(st, nseg, g0);
    const long local = g0 - st->seg[s].start + threadIdx.x;
    if (local >= st->seg[s].total || !as_const(st->active)[st->seg[s].prob]) continue;
    const PassArgs<T> &pa = table_ref(st->seg[s].pa);
    const int mode = st->seg[s].mode;
    switch (st->seg[s].p) {
      case 1: pass_item<T, 1>(mode, local, pa); break;
      case 2: pass_item<T, 2>(mode, local, pa); break;
      case 3: pass_item<T, 3>(mode, local, pa); break;
      case 4: pass_item<T, 4>(mode, local, pa); break;
      case 5: pass_item<T, 5>(mode, local, pa); break;
      case 6: pass_item<T, 6>(mode, local, pa); break;
      case 7: pass_item<T, 7>(mode, local, pa); break;
      case 8: pass_item<T, 8>(mode, local, pa); break;
      default: break;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kCoarseThreads) void k_bcoarse(const BCoarseStage<T> *st_, int lds_elems) {
  const cptr<BCoarseStage<T>> st = as_const(st_);
  if (!as_const(st->active)[st->prob[blockIdx.x]]) return;
  CoarseBody<3, T, kCoarseThreads>::run(threadIdx.x, table_ref(st->seg[blockIdx.x]), lds_arena<double>(), lds_elems);
}

// kind 0: z = 0 on interior nodes, z = r on boundary nodes (in = r, out = z, type T)
// kind 1: out (T) = in (double)            kind 2: out (double) = in (T)
// kind 3: out (double) = in (double)
template <typename T>
__global__ __launch_bounds__(256) void k_belem(const BElemStage *st_) {
  const cptr<BElemStage> st = as_const(st_);
  const int nseg = st->nseg, kind = st->kind;
  const long tot = st->total;
  for (long g0 = (long)blockIdx.x * 256; g0 < tot; g0 += (long)gridDim.x * 256) {
    const int s = seg_of(st, nseg, g0);
    const long i = g0 - st->seg[s].start + threadIdx.x;
    if (i >= st->seg[s].count || !as_const(st->active)[st->seg[s].prob]) continue;
    if (kind == 0) {
      const int m = st->seg[s].m;
      const int x = (int)(i % m), y = (int)((i / m) % m), z = (int)(i / ((long)m * m));
      const bool bnd = x == 0 || x == m - 1 || y == 0 || y == m - 1 || z == 0 || z == m - 1;
      ((T *)st->seg[s].out)[i] = bnd ? ((const T *)st->seg[s].in)[i] : T(0);
    } else if (kind == 1) {
      ((T *)st->seg[s].out)[i] = (T)((const double *)st->seg[s].in)[i];
    } else if (kind == 2) {
      ((double *)st->seg[s].out)[i] = (double)((const T *)st->seg[s].in)[i];
    } else {
      ((double *)st->seg[s].out)[i] = ((const double *)st->seg[s].in)[i];
    }
  }
}

template <typename T>
struct SmoothBytes {
  template <int P>
  struct F {
    static int run(int n_iter, bool one, size_t *o) {
      using B = PatchBody<3, T, patch_threads(P, 3, sizeof(T)), P, typename PaperH<P>::type>;
      *o = (one ? B::arena_one() : B::arena(n_iter)) * sizeof(T);
      return 0;
    }
  };
};

template <typename T>
struct ApplyBytes {
  template <int P>
  struct F {
    static int run(int opt, size_t *o) {
      *o = (opt == 0 ? BMarch<T, P, false>::size : ApplyBody<3, T, apply_threads(P), P, batch_tile(P, 1), false>::size) *
           sizeof(T);
      return 0;
    }
  };
};

int ok() { return hipGetLastError() == hipSuccess ? 0 : -4; }

// ---- batched FCG vectors ----
constexpr int kT = 256;

__device__ inline double block_sum(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// grid = blocks; block b handles chunk b - start of the segment that holds it
__global__ __launch_bounds__(kT) void k_bvec(const BVecStage *st_, int op) {
  __shared__ double sh[kT];
  const cptr<BVecStage> st = as_const(st_);
  const int seg = seg_of(st, st->nseg, blockIdx.x);
  const int bps = st->seg[seg].bps, chunk = blockIdx.x - st->seg[seg].start;
  const long n = st->seg[seg].n;
  const bool act = as_const(st->active)[seg] != 0;
  const double *scal = st->scal + seg * S_COUNT;
  double *part = st->part + 2L * st->seg[seg].start;
  double *x = st->seg[seg].x, *r = st->seg[seg].r, *ro = st->seg[seg].rold, *z = st->seg[seg].z;
  double *p = st->seg[seg].p, *q = st->seg[seg].q;
  if (!act) return;  // uniform per block
  const long stride = (long)bps * kT, i0 = (long)chunk * kT + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  if (op == 0) {
    for (long i = i0; i < n; i += stride) s0 += p[i] * q[i];
  } else if (op == 1) {
    const double alpha = scal[S_ALPHA];
    for (long i = i0; i < n; i += stride) {
      const double ri = r[i];
      x[i] += alpha * p[i];
      ro[i] = ri;
      const double rn = ri - alpha * q[i];
      r[i] = rn;
      s0 += rn * rn;
    }
  } else if (op == 2) {
    for (long i = i0; i < n; i += stride) {
      s0 += z[i] * r[i];
      s1 += z[i] * ro[i];
    }
  } else if (op == 3) {
    const double beta = scal[S_BETA];
    for (long i = i0; i < n; i += stride) p[i] = z[i] + beta * p[i];
    return;
  } else {
    for (long i = i0; i < n; i += stride) s0 += r[i] * r[i];
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    part[chunk] = s0;
    part[bps + chunk] = s1;
  }
}

// one block per segment: sum the partials in a fixed order and update the scalars
__global__ __launch_bounds__(kT) void k_bvec_final(const BVecStage *st_, int op) {
  __shared__ double sh[kT];
  const cptr<BVecStage> st = as_const(st_);
  const int seg = blockIdx.x, bps = st->seg[seg].bps;
  const bool act = as_const(st->active)[seg] != 0;
  double *scal = st->scal + seg * S_COUNT;
  const double *part = st->part + 2L * st->seg[seg].start;
  if (!act) return;  // uniform per block
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < bps; i += kT) {
    a += part[i];
    b += part[bps + i];
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x != 0) return;
  if (op == 0) {
    scal[S_PQ] = a;
    scal[S_ALPHA] = scal[S_RZ] / a;
  } else if (op == 1) {
    scal[S_RR] = a;
  } else if (op == 2) {
    scal[S_ZRN] = a;
    scal[S_ZRO] = b;
    scal[S_BETA] = (a - b) / scal[S_RZ];
    scal[S_RZ] = a;
  } else if (op == 4) {
    scal[S_BB] = a;
    scal[S_RR] = a;
  }
}

}  // namespace

template <typename T>
size_t BatchLaunch<T>::smooth_bytes(int p, int n_iter, bool one) {
  size_t o = 0;
  return dispatch_degree<SmoothBytes<T>::template F>(p, n_iter, one, &o) == 0 ? o : 0;
}

template <typename T>
size_t BatchLaunch<T>::apply_bytes(int p, int tile) {
  size_t o = 0;
  return dispatch_degree<ApplyBytes<T>::template F>(p, tile, &o) == 0 ? o : 0;
}

// Kernel addresses by degree (and tile option, residual mode).
template <typename T>
struct KernelTable {
  template <int P>
  struct F {
    static int run(const void **sm, const void **ap) {
      sm[0] = (const void *)k_bsmooth<T, P, false>;
      sm[1] = (const void *)k_bsmooth<T, P, true>;
      ap[0] = (const void *)k_bmarch<T, P, false>;
      ap[1] = (const void *)k_bmarch<T, P, true>;
      ap[2] = (const void *)k_bapply<T, P, 1, false>;
      ap[3] = (const void *)k_bapply<T, P, 1, true>;
      return 0;
    }
  };
};

template <typename T>
int BatchLaunch<T>::prepare(size_t shmem) {
  if (shmem <= 65536) return 0;
  for (int p = 1; p <= kMaxDegree; ++p) {
    const void *sm[2] = {}, *ap[4] = {};
    if (dispatch_degree<KernelTable<T>::template F>(p, sm, ap) != 0) return -2;
    for (const void *k : {sm[0], sm[1], ap[0], ap[1], ap[2], ap[3]})
      if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem) != hipSuccess) return -4;
  }
  return 0;
}

template <typename T>
int BatchLaunch<T>::smooth(const BSmoothStage<T> *st, int p, bool one, int grid, size_t shmem, hipStream_t s) {
  if (grid <= 0) return 0;
  const void *sm[2] = {}, *ap[4] = {};
  if (dispatch_degree<KernelTable<T>::template F>(p, sm, ap) != 0) return -2;
  void *args[] = {(void *)&st};
  if (hipLaunchKernel(sm[one ? 1 : 0], dim3(grid), dim3(patch_threads(p, 3, sizeof(T))), args, shmem, s) !=
      hipSuccess)
    return -4;
  return 0;
}

template <typename T>
int BatchLaunch<T>::apply(const BApplyStage<T> *st, int p, int tile, bool resid, int grid, size_t shmem,
                          hipStream_t s) {
  if (grid <= 0) return 0;
  const void *sm[2] = {}, *ap[4] = {};
  if (dispatch_degree<KernelTable<T>::template F>(p, sm, ap) != 0) return -2;
  void *args[] = {(void *)&st};
  const int threads = tile != 0 ? apply_threads(p) : march_threads(p);
  if (hipLaunchKernel(ap[2 * (tile != 0) + (resid ? 1 : 0)], dim3(grid), dim3(threads), args, shmem, s) != hipSuccess)
    return -4;
  return 0;
}

template <typename T>
int BatchLaunch<T>::pass(const BPassStage<T> *st, int grid, hipStream_t s) {
  if (grid <= 0) return 0;
  hipLaunchKernelGGL(k_bpass<T>, dim3(grid), dim3(kBatchThreads), 0, s, st);
  return ok();
}

template <typename T>
int BatchLaunch<T>::coarse(const BCoarseStage<T> *st, int nseg, hipStream_t s) {
  if (nseg <= 0) return 0;
  // every segment runs on the device's full LDS; one whose work vectors do not fit it uses
  // its global buffers
  const size_t bytes = device_lds_limit();
  if (bytes > 65536) {
    static thread_local bool raised = false;
    if (!raised) {
      if (hipFuncSetAttribute((const void *)k_bcoarse<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
          hipSuccess)
        return -4;
      raised = true;
    }
  }
  hipLaunchKernelGGL(k_bcoarse<T>, dim3(nseg), dim3(kCoarseThreads), bytes, s, st, (int)(bytes / sizeof(double)));
  return ok();
}

template <typename T>
int BatchLaunch<T>::elem(const BElemStage *st, int grid, hipStream_t s) {
  if (grid <= 0) return 0;
  hipLaunchKernelGGL(k_belem<T>, dim3(grid), dim3(256), 0, s, st);
  return ok();
}

template struct BatchLaunch<double>;
template struct BatchLaunch<float>;

int launch_bvec(const BVecStage *st, int op, int nseg, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_bvec, dim3(blocks), dim3(kT), 0, s, st, op);
  if (hipGetLastError() != hipSuccess) return -4;
  if (op == 3) return 0;
  hipLaunchKernelGGL(k_bvec_final, dim3(nseg), dim3(kT), 0, s, st, op);
  return ok();
}

}  // namespace pmg
