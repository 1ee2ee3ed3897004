// Batched stages: many independent Cartesian 3D problems (different sizes and degrees)
// advance through one V-cycle stage together.  A stage table in device memory (read
// through the constant address space) lists up to kBatchMax segments, one per problem;
// a persistent grid of workgroups walks the concatenated work items (patches, tiles,
// nodes) of all segments.  Patch and apply kernels exist once per degree, shaped like
// the single-problem kernels of that degree (paper p-hierarchy), so a stage with several
// degrees is one launch per degree, the launches independent of each other.
#pragma once

#include <hip/hip_runtime.h>

#include "bodies.h"
#include "constants.h"
#include "dispatch.h"

namespace pmg {

constexpr int kBatchMax = 16;
constexpr int kBatchThreads = 256;  // workgroup size of the batched transfer kernel

// Apply option of a degree: 0 the marching apply of the single-problem path; 1 the owned-node
// tile apply with batch_tile(p, 1) cells per direction (its own tables).  batch_tile(p, 0)
// is the single-problem tile size.
constexpr int batch_tile(int p, int opt) {
  return opt == 0 ? tile_cells(p) : (tile_cells(p) > 1 ? tile_cells(p) - 1 : 1);
}

template <typename T>
struct BSmoothSeg {
  int start, p, prob;  // first work item (patch) of the segment in the stage; degree; problem
  SmoothArgs<T> a;   // one color of one h-level of one problem
};

template <typename T>
struct BSmoothStage {
  int nseg, total;
  const int *active;  // [problem] nonzero while the problem takes part (device array)
  BSmoothSeg<T> seg[kBatchMax];
};

template <typename T>
struct BApplySeg {
  int start, p, prob, tile;  // tile: 0 the default tile of the degree, 1 the alternative
  ApplyArgs<T> a;
};

template <typename T>
struct BApplyStage {
  int nseg, total, resid;
  const int *active;
  BApplySeg<T> seg[kBatchMax];
};

template <typename T>
struct BPassSeg {
  int p, prob;
  int mode;      // 0 restrict, 1 prolong (overwrite), 2 prolong (add)
  long start;    // first thread of the segment, a multiple of kBatchThreads
  long total;
  PassArgs<T> pa;
};

template <typename T>
struct BPassStage {
  int nseg;
  long total_threads;
  const int *active;
  BPassSeg<T> seg[kBatchMax];
};

template <typename T>
struct BCoarseStage {
  int nseg;
  const int *active;
  int prob[kBatchMax];
  CoarseArgs<T> seg[kBatchMax];
};

// elementwise: kind 0 init_z (z = 0 interior, z = r boundary), 1 cast f64->T, 2 cast T->f64
struct BElemSeg {
  long start, count;
  int m, prob;
  const void *in;
  void *out;
  const void *aux;
};

struct BElemStage {
  int nseg, kind;
  long total;
  const int *active;
  BElemSeg seg[kBatchMax];
};

}  // namespace pmg

namespace pmg {

// p-hierarchy type of the paper's rule for each degree
template <int P>
struct PaperH;
template <> struct PaperH<1> { using type = Degrees<1>; };
template <> struct PaperH<2> { using type = Degrees<1, 2>; };
template <> struct PaperH<3> { using type = Degrees<1, 3>; };
template <> struct PaperH<4> { using type = Degrees<1, 3, 4>; };
template <> struct PaperH<5> { using type = Degrees<1, 3, 5>; };
template <> struct PaperH<6> { using type = Degrees<1, 3, 6>; };
template <> struct PaperH<7> { using type = Degrees<1, 3, 7>; };
template <> struct PaperH<8> { using type = Degrees<1, 3, 7, 8>; };

// Launchers (batch.hip).  Stage tables live in device memory (written once when a batch
// is created) and are read through the constant address space.
template <typename T>
struct BatchLaunch {
  // dynamic LDS of the patch kernel (one: the kernel of the default local solver alone)
  static size_t smooth_bytes(int p, int n_iter, bool one = false);
  static size_t apply_bytes(int p, int tile);
  // every segment of a smooth or apply stage table has degree p (one kernel per degree,
  // shaped like the single-problem kernel of that degree); tile: batch_tile option; one:
  // every segment has the default local solver (one half V-cycle, one Richardson step)
  static int smooth(const BSmoothStage<T> *st_dev, int p, bool one, int grid, size_t shmem, hipStream_t s);
  static int apply(const BApplyStage<T> *st_dev, int p, int tile, bool resid, int grid, size_t shmem, hipStream_t s);
  static int pass(const BPassStage<T> *st_dev, int grid, hipStream_t s);
  static int coarse(const BCoarseStage<T> *st_dev, int nseg, hipStream_t s);
  static int elem(const BElemStage *st_dev, int grid, hipStream_t s);
  static int prepare(size_t shmem);  // raise the dynamic LDS limit of the workgroup kernels
};

}  // namespace pmg

namespace pmg {

// ---- batched outer flexible CG (FP64): one segment per problem ----
struct BVecSeg {
  int start, bps;      // first reduction block of the segment, its block count
  long n;
  double *x, *r, *rold, *z, *p, *q;
};

struct BVecStage {
  int nseg, blocks;    // segments (problems), total reduction blocks
  double *part;        // [2 * blocks] partial sums, segment k at 2 * start
  double *scal;        // [seg][S_COUNT] scalars (Scal indices of launch.h)
  const int *active;   // [seg] nonzero while the problem iterates
  BVecSeg seg[kBatchMax];
};

// Vector operation `op` on the segments whose active flag is set (the others are left
// untouched), with deterministic fixed-tree reductions:
//  0: pq = (p, q); alpha = rz / pq
//  1: x += alpha p, rold = r, r -= alpha q; rr = (r, r)
//  2: zrn = (z, r), zro = (z, rold); beta = (zrn - zro) / rz; rz = zrn
//  3: p = z + beta p
//  4: bb = rr = (r, r)
int launch_bvec(const BVecStage *st_dev, int op, int nseg, int blocks, hipStream_t s);

}  // namespace pmg
