// Batches of independent problems (declared in include/pmg.h): stage tables of the
// depth-aligned V-cycle, their launch on one stream with class-parallel branches, HIP
// graph capture, the batched outer flexible CG, and the launch-parameter tuner with its
// cache file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <exception>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "batch.h"
#include "dispatch.h"
#include "problem.h"

using namespace pmg;

namespace {

constexpr int kLanes = kMaxDegree;  // independent launches of one stage: one per degree

enum Kind { K_SMOOTH = 0, K_APPLY, K_PASS, K_COARSE, K_ELEM };

// One launch.  Consecutive steps with the same group touch disjoint problems and may run
// concurrently.
struct Step {
  int kind = 0, p = 0, tile = 0, resid = 0, group = 0;  // p: degree of smooth and apply steps
  int one = 0;  // smooth step whose segments all have the default local solver
  size_t off = 0;    // byte offset of the stage table in the plan's device buffer
  long items = 0;    // workgroups of work: patches, tiles, or 256-thread blocks
  size_t shmem = 0;  // dynamic LDS of the launch
  int grid = 0;
};

// Launch parameters of one plan: persistent workgroups per compute unit of each kernel
// (0: one workgroup per work item) and the apply tile option, per degree.
struct Tuning {
  // the launches of one stage (one per degree) run as parallel branches when the stage has at
  // most this many work items in all, else one after another: a launch that fills the GPU by
  // itself only competes for compute units and caches with the ones beside it
  int lane_items = 4096;
  int smooth_wpc[kMaxDegree + 1] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int apply_wpc[kMaxDegree + 1] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int pass_wpc = 0, elem_wpc = 0;
  int tile[kMaxDegree + 1] = {};
};

template <typename T>
struct Plan {
  bool supported = false;
  bool pending = false;  // some launch parameter still has to be measured
  std::vector<Step> steps;
  std::vector<unsigned char> blob;  // host image of the stage tables
  unsigned char *dev = nullptr;     // device copy
  size_t cap = 0;
  Tuning tune;
  hipGraphExec_t vgraph = nullptr;  // one V-cycle
  hipGraphExec_t igraph = nullptr;  // one outer CG iteration (V-cycle + vector updates + apply)
};

}  // namespace

struct pmg_batch {
  int n = 0, device = -1, ncu = 256;
  size_t lds_max = 0;
  std::string arch, cache_path;
  std::map<std::string, int> cache;  // launch parameters by "arch/3d/precision/knob"
  std::vector<pmg_problem *> pr;
  Plan<double> p64;   // multigrid in float64
  Plan<float> p32;    // multigrid in float32
  Plan<double> outer; // operator apply of the outer CG (float64)
  // alternative apply-tile tables per problem
  std::vector<const double *> kt64, mt64;
  std::vector<const float *> kt32, mt32;
  std::vector<void *> allocs;
  int *active = nullptr, *hactive = nullptr;  // [n] device flags and their pinned mirror
  double *part = nullptr, *scal = nullptr, *hscal = nullptr;
  BVecStage *vec = nullptr, *hvec = nullptr;  // outer CG vector table, device and pinned
  int vec_blocks = 0;
  hipStream_t cs = nullptr, aux[kLanes - 1] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kLanes - 1] = {}, t0 = nullptr, t1 = nullptr;
};

namespace {

// ---- device buffers owned by the batch ----
template <typename T>
int balloc(pmg_batch *bt, T **out, size_t count) {
  void *ptr = nullptr;
  PMG_HIP(hipMalloc(&ptr, count * sizeof(T) + 64));
  bt->allocs.push_back(ptr);
  *out = reinterpret_cast<T *>(ptr);
  return PMG_OK;
}

template <typename T>
T *fin_r(pmg_problem *pr);
template <>
double *fin_r<double>(pmg_problem *pr) { return pr->fr[0]; }
template <>
float *fin_r<float>(pmg_problem *pr) { return pr->d32.r[pr->finest()]; }
template <typename T>
T *fin_z(pmg_problem *pr);
template <>
double *fin_z<double>(pmg_problem *pr) { return pr->fz; }
template <>
float *fin_z<float>(pmg_problem *pr) { return pr->d32.z[pr->finest()]; }

// V-cycle vectors of h-level l: right-hand side and correction.  On the finest level the
// float64 cycle works on the outer CG's residual and preconditioned residual directly.
template <typename T>
T *vec_r(pmg_problem *pr, int l) { return l == pr->finest() ? fin_r<T>(pr) : pr->pd<T>().r[l]; }
template <typename T>
T *vec_z(pmg_problem *pr, int l) { return l == pr->finest() ? fin_z<T>(pr) : pr->pd<T>().z[l]; }

template <typename T>
const T *alt_kt(pmg_batch *bt, int i);
template <>
const double *alt_kt<double>(pmg_batch *bt, int i) { return bt->kt64[i]; }
template <>
const float *alt_kt<float>(pmg_batch *bt, int i) { return bt->kt32[i]; }
template <typename T>
const T *alt_mt(pmg_batch *bt, int i);
template <>
const double *alt_mt<double>(pmg_batch *bt, int i) { return bt->mt64[i]; }
template <>
const float *alt_mt<float>(pmg_batch *bt, int i) { return bt->mt32[i]; }

// Appends the used part of a stage table (header + nseg segments), 256-byte aligned.
template <typename S>
size_t put(std::vector<unsigned char> &blob, const S &st, size_t bytes) {
  const size_t off = (blob.size() + 255) / 256 * 256;
  blob.resize(off + bytes);
  std::memcpy(blob.data() + off, &st, bytes);
  return off;
}

template <typename S, typename Seg>
size_t used_bytes(int nseg) {
  return offsetof(S, seg) + (size_t)nseg * sizeof(Seg);
}

long round256(long x) { return (x + 255) / 256 * 256; }

// Work items of a segment start at a multiple of 8: with a grid that is a multiple of 8,
// work item i then runs on XCD i mod 8 as in a single-problem launch, which is what the
// XCD-aware patch and tile order of the kernel bodies assumes.
int round8(int x) { return (x + 7) / 8 * 8; }

// ---- plan construction ----
template <typename T>
struct Builder {
  pmg_batch *bt;
  Plan<T> &pl;
  int group = 0;

  void push(int kind, int p, int tile, int resid, size_t off, long items, size_t shmem) {
    Step s;
    s.kind = kind;
    s.p = p;
    s.tile = tile;
    s.resid = resid;
    s.group = group;
    s.off = off;
    s.items = items;
    s.shmem = shmem;
    pl.steps.push_back(s);
  }

  // elementwise stage over the listed (problem, level) pairs
  void elem(int kind, const std::vector<std::pair<int, int>> &parts) {
    BElemStage st{};
    st.kind = kind;
    st.active = bt->active;
    long tot = 0;
    for (auto [i, l] : parts) {
      pmg_problem *pr = bt->pr[i];
      const int L = pr->finest();
      BElemSeg &g = st.seg[st.nseg++];
      g.start = tot;
      g.count = pr->nodes(l);
      g.m = pr->p * pr->sizes[l] + 1;
      g.prob = i;
      if (kind == 0) {
        g.in = vec_r<T>(pr, l);
        g.out = vec_z<T>(pr, l);
      } else if (kind == 1) {
        g.in = pr->fr[0];
        g.out = fin_r<T>(pr);
      } else {
        g.in = fin_z<T>(pr);
        g.out = pr->fz;
      }
      (void)L;
      tot += round256(g.count);
    }
    if (!st.nseg) return;
    st.total = tot;
    push(K_ELEM, 0, 0, 0, put(pl.blob, st, used_bytes<BElemStage, BElemSeg>(st.nseg)), tot / 256, 0);
    ++group;
  }

  // one color sweep stage over the listed (problem, level) pairs
  void smooth(const std::vector<std::pair<int, int>> &parts, int col) {
    BSmoothStage<T> st[kLanes + 1]{};
    int tot[kLanes + 1] = {};
    for (auto [i, l] : parts) {
      pmg_problem *pr = bt->pr[i];
      const int n = pr->sizes[l], p = pr->p;
      SmoothArgs<T> a{};
      a.tb = pr->pd<T>().tabs;
      a.c = (T)pr->cscale(l);
      a.cinv = (T)(1.0 / pr->cscale(l));
      a.n = n;
      a.full = pr->cfg.local_solver == PMG_LOCAL_FULL_V;
      a.n_iter = pr->cfg.n_local_iter;
      a.direct = pr->cfg.local_solver == PMG_LOCAL_DIRECT;
      a.reinf = pr->cfg.local_smoother == PMG_SMOOTHER_REINFORCED;
      for (int q = 0; q < pr->nplev() && q < 4; ++q) a.om.w[q] = (T)pr->tab.omega[q];
      a.u = vec_z<T>(pr, l);
      a.b = vec_r<T>(pr, l);
      a.n_patch = 1;
      for (int d = 0; d < 3; ++d) {
        a.first[d] = (col >> d) & 1 ? 1 : 2;
        a.cnt[d] = a.first[d] <= n - 1 ? (n - 1 - a.first[d]) / 2 + 1 : 0;
        a.n_patch *= a.cnt[d];
      }
      if (a.n_patch == 0) continue;
      BSmoothSeg<T> &g = st[p].seg[st[p].nseg++];
      g.start = tot[p];
      g.p = p;
      g.prob = i;
      g.a = a;
      tot[p] += round8(a.n_patch);
    }
    bool any = false;
    for (int p = 1; p <= kLanes; ++p) {
      if (!st[p].nseg) continue;
      st[p].total = tot[p];
      st[p].active = bt->active;
      int iters = 1;
      bool one = true;
      for (int k = 0; k < st[p].nseg; ++k) {
        const SmoothArgs<T> &a = st[p].seg[k].a;
        iters = std::max(iters, a.n_iter);
        one = one && a.full == 0 && a.n_iter == 1 && a.direct == 0 && a.reinf == 0;
      }
      push(K_SMOOTH, p, 0, 0, put(pl.blob, st[p], used_bytes<BSmoothStage<T>, BSmoothSeg<T>>(st[p].nseg)), tot[p],
           BatchLaunch<T>::smooth_bytes(p, iters, one));
      pl.steps.back().one = one;
      any = true;
    }
    if (any) ++group;
  }

  // operator apply on h-level l of each listed problem: residual (out = t_l = R - A Z) in
  // the V-cycle, or q = A p of the outer CG
  void apply(const std::vector<std::pair<int, int>> &parts, bool resid) {
    BApplyStage<T> st[kLanes + 1]{};
    int tot[kLanes + 1] = {};
    for (auto [i, l] : parts) {
      pmg_problem *pr = bt->pr[i];
      const int p = pr->p, opt = pl.tune.tile[p];
      ApplyArgs<T> a{};
      a.Kt = opt ? alt_kt<T>(bt, i) : pr->pd<T>().tabs.Kt;
      a.Mt = opt ? alt_mt<T>(bt, i) : pr->pd<T>().tabs.Mt;
      a.c = (T)pr->cscale(l);
      a.n = pr->sizes[l];
      if (opt == 0) {  // the marching apply, with the single-problem launch geometry
        int nz;
        march_geometry(a.n, march_tile(p), march_tile_y(p), kMarchBlocks, a.mt, a.mty, nz, a.zc);
        a.n_tiles = a.mt * a.mty * nz;
      } else {
        const int tc = batch_tile(p, opt);
        a.ntile = (a.n + tc - 1) / tc;
        a.n_tiles = a.ntile * a.ntile * a.ntile;
      }
      if (resid) {
        a.u = vec_z<T>(pr, l);
        a.b = vec_r<T>(pr, l);
        a.out = pr->pd<T>().t[l];
      } else if constexpr (std::is_same<T, double>::value) {
        a.u = pr->fp;
        a.b = nullptr;
        a.out = pr->fq;
      }
      BApplySeg<T> &g = st[p].seg[st[p].nseg++];
      g.start = tot[p];
      g.p = p;
      g.prob = i;
      g.tile = opt;
      g.a = a;
      tot[p] += round8(a.n_tiles);
    }
    bool any = false;
    for (int p = 1; p <= kLanes; ++p) {
      if (!st[p].nseg) continue;
      st[p].total = tot[p];
      st[p].resid = resid;
      st[p].active = bt->active;
      push(K_APPLY, p, pl.tune.tile[p], resid,
           put(pl.blob, st[p], used_bytes<BApplyStage<T>, BApplySeg<T>>(st[p].nseg)), tot[p],
           BatchLaunch<T>::apply_bytes(p, pl.tune.tile[p]));
      any = true;
    }
    if (any) ++group;
  }

  // the three 1D passes of the h-transfer between level l and l-1 of each listed problem
  void transfer(const std::vector<std::pair<int, int>> &parts, bool restrict_) {
    if (parts.empty()) return;
    BPassStage<T> st[3]{};
    long thr[3] = {0, 0, 0};
    for (auto [i, l] : parts) {
      pmg_problem *pr = bt->pr[i];
      TransferArgs<T> ta{};
      ta.W1 = pr->pd<T>().tabs.W1;
      ta.Wr = pr->pd<T>().tabs.Wr;
      ta.nc = pr->sizes[l - 1];
      ta.in = restrict_ ? pr->pd<T>().t[l] : vec_z<T>(pr, l - 1);
      ta.out = restrict_ ? vec_r<T>(pr, l - 1) : vec_z<T>(pr, l);
      ta.w1 = pr->pd<T>().tw1;
      ta.w2 = pr->pd<T>().tw2;
      PassArgs<T> pa[3];
      transfer_passes<T>(3, pr->p, restrict_, ta, pa);
      for (int k = 0; k < 3; ++k) {
        BPassSeg<T> &g = st[k].seg[st[k].nseg++];
        g.p = pr->p;
        g.prob = i;
        g.mode = restrict_ ? 0 : (k == 2 ? 2 : 1);
        g.start = thr[k];
        g.total = (long)pa[k].oe[0] * pa[k].oe[1] * pa[k].oe[2];
        g.pa = pa[k];
        thr[k] += round256(g.total);
      }
    }
    for (int k = 0; k < 3; ++k) {
      st[k].total_threads = thr[k];
      st[k].active = bt->active;
      push(K_PASS, 0, 0, 0, put(pl.blob, st[k], used_bytes<BPassStage<T>, BPassSeg<T>>(st[k].nseg)), thr[k] / 256,
           0);
      ++group;
    }
  }

  void coarse() {
    BCoarseStage<T> st{};
    st.active = bt->active;
    for (int i = 0; i < bt->n; ++i) {
      pmg_problem *pr = bt->pr[i];
      CoarseArgs<T> a{};
      a.S = pr->S0;
      a.lam = pr->lam0;
      a.c0inv = 1.0 / pr->cscale(0);
      a.m = pr->tab.m0;
      a.mt = pr->tab.m0 + 2;
      a.r = vec_r<T>(pr, 0);
      a.z = vec_z<T>(pr, 0);
      a.w1 = pr->cw1;
      a.w2 = pr->cw2;
      st.prob[st.nseg] = i;
      st.seg[st.nseg++] = a;
    }
    push(K_COARSE, 0, 0, 0, put(pl.blob, st, used_bytes<BCoarseStage<T>, CoarseArgs<T>>(st.nseg)), st.nseg, 0);
    ++group;
  }
};

// (problem, level) pairs at depth d below the finest level that still have a coarser level
std::vector<std::pair<int, int>> at_depth(pmg_batch *bt, int d) {
  std::vector<std::pair<int, int>> v;
  for (int i = 0; i < bt->n; ++i) {
    const int l = bt->pr[i]->finest() - d;
    if (l >= 1) v.push_back({i, l});
  }
  return v;
}

// V-cycle of every problem (Sec. 2: pre-smoothing, residual and restriction from the
// finest level down, the coarse solve, prolongation and post-smoothing back up), stages
// aligned by depth below each problem's finest level.
template <typename T>
void build_vcycle(pmg_batch *bt, Plan<T> &pl) {
  pl.steps.clear();
  pl.blob.clear();
  Builder<T> b{bt, pl};
  int depth = 0, npre = 0, npost = 0;
  for (pmg_problem *pr : bt->pr) {
    depth = std::max(depth, pr->finest());
    npre = std::max(npre, pr->cfg.n_pre);
    npost = std::max(npost, pr->cfg.n_post);
  }
  std::vector<std::pair<int, int>> fin;
  for (int i = 0; i < bt->n; ++i) fin.push_back({i, bt->pr[i]->finest()});
  if (std::is_same<T, float>::value) b.elem(1, fin);
  for (int d = 0; d < depth; ++d) {
    const auto parts = at_depth(bt, d);
    b.elem(0, parts);
    for (int k = 0; k < npre; ++k) {
      std::vector<std::pair<int, int>> sw;
      for (auto pl_ : parts)
        if (k < bt->pr[pl_.first]->cfg.n_pre) sw.push_back(pl_);
      for (int col = 0; col < 8; ++col) b.smooth(sw, col);
    }
    b.apply(parts, true);
    b.transfer(parts, true);
  }
  b.coarse();
  for (int d = depth - 1; d >= 0; --d) {
    const auto parts = at_depth(bt, d);
    b.transfer(parts, false);
    for (int k = 0; k < npost; ++k) {
      std::vector<std::pair<int, int>> sw;
      for (auto pl_ : parts)
        if (k < bt->pr[pl_.first]->cfg.n_post) sw.push_back(pl_);
      for (int col = 7; col >= 0; --col) b.smooth(sw, col);
    }
  }
  if (std::is_same<T, float>::value) b.elem(2, fin);
}

void build_outer(pmg_batch *bt, Plan<double> &pl) {
  pl.steps.clear();
  pl.blob.clear();
  Builder<double> b{bt, pl};
  std::vector<std::pair<int, int>> fin;
  for (int i = 0; i < bt->n; ++i) fin.push_back({i, bt->pr[i]->finest()});
  b.apply(fin, false);
}

template <typename T>
void size_grids(pmg_batch *bt, Plan<T> &pl) {
  for (Step &s : pl.steps) {
    int wpc = 0;
    switch (s.kind) {
      case K_SMOOTH: wpc = pl.tune.smooth_wpc[s.p]; break;
      case K_APPLY: wpc = pl.tune.apply_wpc[s.p]; break;
      case K_PASS: wpc = pl.tune.pass_wpc; break;
      case K_ELEM: wpc = pl.tune.elem_wpc; break;
      default: wpc = 0;
    }
    long g = s.items;
    if (wpc > 0) g = std::min(g, (long)wpc * bt->ncu / 8 * 8);
    s.grid = (int)std::max(1L, g);
  }
}

template <typename T>
void drop_graphs(Plan<T> &pl) {
  if (pl.vgraph) (void)hipGraphExecDestroy(pl.vgraph);
  if (pl.igraph) (void)hipGraphExecDestroy(pl.igraph);
  pl.vgraph = pl.igraph = nullptr;
}

// (Re)builds the tables of a plan from its tuning and uploads them.
template <typename T>
int upload(pmg_batch *bt, Plan<T> &pl, bool outer) {
  if constexpr (std::is_same<T, double>::value) {
    if (outer)
      build_outer(bt, pl);
    else
      build_vcycle<T>(bt, pl);
  } else {
    build_vcycle<T>(bt, pl);
  }
  size_grids(bt, pl);
  // the captured graphs hold launch shapes: every graph that contains these steps goes
  drop_graphs(bt->p64);
  drop_graphs(bt->p32);
  drop_graphs(bt->outer);
  if (pl.blob.size() > pl.cap) {
    void *p = nullptr;
    PMG_HIP(hipMalloc(&p, pl.blob.size()));
    bt->allocs.push_back(p);
    pl.dev = (unsigned char *)p;
    pl.cap = pl.blob.size();
  }
  PMG_HIP(hipMemcpy(pl.dev, pl.blob.data(), pl.blob.size(), hipMemcpyHostToDevice));
  return PMG_OK;
}

// ---- execution ----
template <typename T>
int launch_step(const Plan<T> &pl, const Step &s, hipStream_t st) {
  const void *tab = pl.dev + s.off;
  switch (s.kind) {
    case K_SMOOTH: return BatchLaunch<T>::smooth((const BSmoothStage<T> *)tab, s.p, s.one != 0, s.grid, s.shmem, st);
    case K_APPLY:
      return BatchLaunch<T>::apply((const BApplyStage<T> *)tab, s.p, s.tile, s.resid, s.grid, s.shmem, st);
    case K_PASS: return BatchLaunch<T>::pass((const BPassStage<T> *)tab, s.grid, st);
    case K_COARSE: return BatchLaunch<T>::coarse((const BCoarseStage<T> *)tab, s.grid, st);
    default: return BatchLaunch<T>::elem((const BElemStage *)tab, s.grid, st);
  }
}

// Launches the steps selected by `keep` in order; the steps of one group after the
// first run on the auxiliary streams, forked from and joined back into `st`.
template <typename T>
int run_steps(pmg_batch *bt, const Plan<T> &pl, hipStream_t st, const std::function<bool(const Step &)> &keep) {
  const auto &v = pl.steps;
  size_t i = 0;
  while (i < v.size()) {
    size_t j = i;
    std::vector<const Step *> grp;
    while (j < v.size() && v[j].group == v[i].group) {
      if (!keep || keep(v[j])) grp.push_back(&v[j]);
      ++j;
    }
    long items = 0;
    for (const Step *g : grp) items += g->items;
    if (grp.size() == 1 || items > pl.tune.lane_items) {
      for (const Step *g : grp) PMG_TRY(launch_step(pl, *g, st));
    } else {
      PMG_HIP(hipEventRecord(bt->ev_fork, st));
      for (size_t k = 1; k < grp.size(); ++k) {
        PMG_HIP(hipStreamWaitEvent(bt->aux[k - 1], bt->ev_fork, 0));
        PMG_TRY(launch_step(pl, *grp[k], bt->aux[k - 1]));
        PMG_HIP(hipEventRecord(bt->ev_join[k - 1], bt->aux[k - 1]));
      }
      PMG_TRY(launch_step(pl, *grp[0], st));
      for (size_t k = 1; k < grp.size(); ++k) PMG_HIP(hipStreamWaitEvent(st, bt->ev_join[k - 1], 0));
    }
    i = j;
  }
  return PMG_OK;
}

int vec_op(pmg_batch *bt, int op, hipStream_t s) {
  PMG_TRY(launch_bvec(bt->vec, op, bt->n, bt->vec_blocks, s));
  return PMG_OK;
}

// One outer CG iteration (Alg. of the flexible CG in pmg_solve, reordered so that the
// preconditioner comes first): z = V(r); beta; p = z + beta p; q = A p; alpha;
// x += alpha p, rold = r, r -= alpha q; (r, r).
template <typename T>
int iteration(pmg_batch *bt, Plan<T> &pl, hipStream_t s) {
  if (int rc = run_steps(bt, pl, s, nullptr)) return rc;
  if (int rc = vec_op(bt, 2, s)) return rc;
  if (int rc = vec_op(bt, 3, s)) return rc;
  if (int rc = run_steps(bt, bt->outer, s, nullptr)) return rc;
  if (int rc = vec_op(bt, 0, s)) return rc;
  return vec_op(bt, 1, s);
}

// Captures `body` on the batch's capture stream into an executable graph.
int capture(pmg_batch *bt, const std::function<int(hipStream_t)> &body, hipGraphExec_t *out) {
  PMG_HIP(hipStreamBeginCapture(bt->cs, hipStreamCaptureModeThreadLocal));
  const int rc = body(bt->cs);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(bt->cs, &g);
  if (rc != PMG_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(PMG_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
  const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return fail(PMG_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
  return PMG_OK;
}

template <typename T>
int ensure_graphs(pmg_batch *bt, Plan<T> &pl) {
  if (!pl.vgraph) {
    if (int rc = capture(bt, [&](hipStream_t s) { return run_steps(bt, pl, s, nullptr); }, &pl.vgraph)) return rc;
  }
  if (!pl.igraph) {
    if (int rc = capture(bt, [&](hipStream_t s) { return iteration(bt, pl, s); }, &pl.igraph)) return rc;
  }
  return PMG_OK;
}

// ---- tuner ----
// Average time of the selected steps (2 runs after one warm-up run), in ms.
template <typename T>
float time_steps(pmg_batch *bt, Plan<T> &pl, const std::function<bool(const Step &)> &keep) {
  if (run_steps(bt, pl, bt->cs, keep) != PMG_OK) return 1e30f;
  if (hipEventRecord(bt->t0, bt->cs) != hipSuccess) return 1e30f;
  for (int r = 0; r < 2; ++r)
    if (run_steps(bt, pl, bt->cs, keep) != PMG_OK) return 1e30f;
  if (hipEventRecord(bt->t1, bt->cs) != hipSuccess || hipEventSynchronize(bt->t1) != hipSuccess) return 1e30f;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, bt->t0, bt->t1) != hipSuccess) return 1e30f;
  return ms / 2.f;
}

struct Knob {
  std::string key;
  int *val;
  std::vector<int> cand;
  std::function<bool(const Step &)> keep;
  bool tables;  // the knob changes stage tables (apply tile)
};

// Every knob is judged by the time of the whole plan (the V-cycle, or the outer apply), so
// that launches of other degrees running beside it count.
template <typename T>
std::vector<Knob> knobs(pmg_batch *bt, Plan<T> &pl, bool outer) {
  std::vector<Knob> k;
  bool deg[kMaxDegree + 1] = {};
  for (pmg_problem *pr : bt->pr) deg[pr->p] = true;
  const std::vector<int> wpc = {0, 1, 2, 4, 8};
  k.push_back({"lane_items", &pl.tune.lane_items, {0, 1024, 4096, 16384, 1 << 30}, nullptr, false});
  for (int p = 1; p <= kMaxDegree; ++p) {
    if (!deg[p]) continue;
    const std::string d = "/p" + std::to_string(p);
    if (!outer) k.push_back({"smooth_wpc" + d, &pl.tune.smooth_wpc[p], wpc, nullptr, false});
    if (BatchLaunch<T>::apply_bytes(p, 1) <= bt->lds_max)
      k.push_back({"apply_tile" + d, &pl.tune.tile[p], {0, 1}, nullptr, true});
    k.push_back({"apply_wpc" + d, &pl.tune.apply_wpc[p], wpc, nullptr, false});
  }
  if (!outer) {
    k.push_back({"pass_wpc", &pl.tune.pass_wpc, {0, 4, 16}, nullptr, false});
    k.push_back({"elem_wpc", &pl.tune.elem_wpc, {0, 4, 16}, nullptr, false});
  }
  return k;
}

// Flat JSON object of string keys and integer values.
std::map<std::string, int> read_cache(const std::string &path) {
  std::map<std::string, int> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = s.substr(i + 1, j - i - 1);
    size_t c = s.find(':', j);
    if (c == std::string::npos) break;
    char *end = nullptr;
    const long v = std::strtol(s.c_str() + c + 1, &end, 10);
    if (end != s.c_str() + c + 1) m[key] = (int)v;
    i = end ? (size_t)(end - s.c_str()) : j + 1;
  }
  return m;
}

int write_cache(const std::string &path, const std::map<std::string, int> &m) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return fail(PMG_ERR_INVALID_ARG, "cannot write tuning cache %s", path.c_str());
    f << "{\n";
    size_t k = 0;
    for (const auto &kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++k < m.size() ? ",\n" : "\n");
    f << "}\n";
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0)
    return fail(PMG_ERR_INVALID_ARG, "cannot write tuning cache %s", path.c_str());
  return PMG_OK;
}

// Takes each knob's value from the cache; with `measure`, times the candidates of the
// knobs the cache lacks, one knob at a time (coordinate descent in the order of `knobs`),
// and records the best.  Otherwise a missing knob keeps its default and the plan stays
// pending.  Measuring runs the plan on the problems' work buffers, zeroed first.
template <typename T>
int tune(pmg_batch *bt, Plan<T> &pl, const std::string &prefix, bool outer, bool measure) {
  std::vector<Knob> ks = knobs(bt, pl, outer);
  std::vector<Knob *> todo;
  for (Knob &k : ks) {
    auto it = bt->cache.find(prefix + k.key);
    if (it != bt->cache.end() && std::find(k.cand.begin(), k.cand.end(), it->second) != k.cand.end())
      *k.val = it->second;
    else
      todo.push_back(&k);
  }
  if (int rc = upload(bt, pl, outer)) return rc;
  pl.pending = !todo.empty();
  if (!measure || todo.empty()) return PMG_OK;
  for (pmg_problem *pr : bt->pr) {
    const size_t N = (size_t)pr->nodes(pr->finest());
    PMG_HIP(hipMemsetAsync(pr->fr[0], 0, N * sizeof(double), bt->cs));
    PMG_HIP(hipMemsetAsync(pr->fp, 0, N * sizeof(double), bt->cs));
  }
  for (Knob *k : todo) {
    int best = *k->val;
    float tbest = 1e30f;
    for (int v : k->cand) {
      *k->val = v;
      if (k->tables) {
        if (int rc = upload(bt, pl, outer)) return rc;
      } else {
        size_grids(bt, pl);
      }
      const float t = time_steps(bt, pl, k->keep);
      if (t < tbest) {
        tbest = t;
        best = v;
      }
    }
    *k->val = best;
    if (k->tables) {
      if (int rc = upload(bt, pl, outer)) return rc;
    } else {
      size_grids(bt, pl);
    }
    bt->cache[prefix + k->key] = best;
  }
  PMG_HIP(hipStreamSynchronize(bt->cs));
  pl.pending = false;
  return write_cache(bt->cache_path, bt->cache);
}

// Before the first use of a plan: measure the knobs its cache entries lack.
template <typename T>
int ready(pmg_batch *bt, Plan<T> &pl, const char *prec, bool outer) {
  if (!pl.pending || bt->cache_path.empty()) return PMG_OK;
  return tune(bt, pl, bt->arch + "/3d/" + prec + "/", outer, true);
}

int check_mg(pmg_batch *bt, int mg_prec) {
  if (mg_prec != PMG_FP64 && mg_prec != PMG_FP32 && mg_prec != PMG_FP32_BF16)
    return fail(PMG_ERR_INVALID_ARG, "precision %d unknown", mg_prec);
  if (mg_prec == PMG_FP64 && !bt->p64.supported)
    return fail(PMG_ERR_UNSUPPORTED, "float64 multigrid: a patch arena of this batch exceeds the LDS");
  return PMG_OK;
}

void destroy(pmg_batch *bt) {
  drop_graphs(bt->p64);
  drop_graphs(bt->p32);
  drop_graphs(bt->outer);
  for (void *p : bt->allocs) (void)hipFree(p);
  if (bt->hactive) (void)hipHostFree(bt->hactive);
  if (bt->hscal) (void)hipHostFree(bt->hscal);
  if (bt->hvec) (void)hipHostFree(bt->hvec);
  if (bt->cs) (void)hipStreamDestroy(bt->cs);
  for (hipStream_t s : bt->aux)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : bt->ev_join)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : {bt->ev_fork, bt->t0, bt->t1})
    if (e) (void)hipEventDestroy(e);
  delete bt;
}

int create(pmg_batch *bt, pmg_problem *const *problems, int n, const char *path) {
  for (int i = 0; i < n; ++i) {
    pmg_problem *pr = problems[i];
    if (!pr) return fail(PMG_ERR_INVALID_ARG, "problem %d is NULL", i);
    for (int j = 0; j < i; ++j)
      if (problems[j] == pr) return fail(PMG_ERR_INVALID_ARG, "problem %d appears twice", i);
    if (!pr->dev) return fail(PMG_ERR_INVALID_ARG, "problem %d: pmg_device_init has not been called", i);
    if (pr->dim != 3) return fail(PMG_ERR_UNSUPPORTED, "problem %d: batches hold 3D problems only", i);
    if (pr->general) return fail(PMG_ERR_UNSUPPORTED, "problem %d: batches hold Cartesian problems only", i);
    if (pr->hcode != 0) return fail(PMG_ERR_UNSUPPORTED, "problem %d: batches use the paper's p-hierarchy only", i);
    if (i > 0 && pr->device != problems[0]->device)
      return fail(PMG_ERR_INVALID_ARG, "problem %d lives on another device", i);
    bt->pr.push_back(pr);
  }
  bt->n = n;
  bt->device = problems[0]->device;
  PMG_HIP(hipSetDevice(bt->device));
  int lds = 0, ncu = 0;
  PMG_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, bt->device));
  PMG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, bt->device));
  bt->lds_max = (size_t)lds;
  bt->ncu = ncu > 0 ? ncu : 256;
  hipDeviceProp_t prop;
  PMG_HIP(hipGetDeviceProperties(&prop, bt->device));
  bt->arch = prop.gcnArchName;
  bt->arch = bt->arch.substr(0, bt->arch.find(':'));
  // which multigrid precisions fit: every patch and apply arena in LDS
  bt->p64.supported = bt->p32.supported = bt->outer.supported = true;
  for (pmg_problem *pr : bt->pr) {
    const int it = pr->cfg.n_local_iter;
    if (BatchLaunch<double>::smooth_bytes(pr->p, it) > bt->lds_max ||
        BatchLaunch<double>::apply_bytes(pr->p, 0) > bt->lds_max)
      bt->p64.supported = false;
    if (BatchLaunch<float>::smooth_bytes(pr->p, it) > bt->lds_max ||
        BatchLaunch<float>::apply_bytes(pr->p, 0) > bt->lds_max)
      bt->p32.supported = false;
    if (BatchLaunch<double>::apply_bytes(pr->p, 0) > bt->lds_max) bt->outer.supported = false;
  }
  if (!bt->p32.supported || !bt->outer.supported)
    return fail(PMG_ERR_UNSUPPORTED, "a kernel arena of this batch exceeds the LDS of the device");
  PMG_TRY(BatchLaunch<double>::prepare(bt->lds_max));
  PMG_TRY(BatchLaunch<float>::prepare(bt->lds_max));
  // streams and events (default priority)
  PMG_HIP(hipStreamCreateWithFlags(&bt->cs, hipStreamNonBlocking));
  for (auto &s : bt->aux) PMG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  PMG_HIP(hipEventCreateWithFlags(&bt->ev_fork, hipEventDisableTiming));
  for (auto &e : bt->ev_join) PMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  PMG_HIP(hipEventCreate(&bt->t0));
  PMG_HIP(hipEventCreate(&bt->t1));
  // alternative apply tiles
  for (pmg_problem *pr : bt->pr) {
    dvec Kt, Mt;
    apply_tile_tables(pr->p, batch_tile(pr->p, 1), Kt, Mt);
    double *k64, *m64;
    float *k32, *m32;
    int rc;
    if ((rc = balloc(bt, &k64, Kt.size())) || (rc = balloc(bt, &m64, Mt.size())) ||
        (rc = balloc(bt, &k32, Kt.size())) || (rc = balloc(bt, &m32, Mt.size())))
      return rc;
    std::vector<float> k32h(Kt.begin(), Kt.end()), m32h(Mt.begin(), Mt.end());
    PMG_HIP(hipMemcpy(k64, Kt.data(), Kt.size() * sizeof(double), hipMemcpyHostToDevice));
    PMG_HIP(hipMemcpy(m64, Mt.data(), Mt.size() * sizeof(double), hipMemcpyHostToDevice));
    PMG_HIP(hipMemcpy(k32, k32h.data(), k32h.size() * sizeof(float), hipMemcpyHostToDevice));
    PMG_HIP(hipMemcpy(m32, m32h.data(), m32h.size() * sizeof(float), hipMemcpyHostToDevice));
    bt->kt64.push_back(k64);
    bt->mt64.push_back(m64);
    bt->kt32.push_back(k32);
    bt->mt32.push_back(m32);
  }
  // outer CG state
  int rc;
  if ((rc = balloc(bt, &bt->active, (size_t)n)) || (rc = balloc(bt, &bt->scal, (size_t)n * S_COUNT)) ||
      (rc = balloc(bt, &bt->vec, 1)))
    return rc;
  PMG_HIP(hipHostMalloc((void **)&bt->hactive, (size_t)n * sizeof(int), hipHostMallocDefault));
  PMG_HIP(hipHostMalloc((void **)&bt->hscal, (size_t)n * S_COUNT * sizeof(double), hipHostMallocDefault));
  PMG_HIP(hipHostMalloc((void **)&bt->hvec, sizeof(BVecStage), hipHostMallocDefault));
  std::memset(bt->hvec, 0, sizeof(BVecStage));
  int blocks = 0;
  for (int i = 0; i < n; ++i) {
    pmg_problem *pr = bt->pr[i];
    BVecSeg &g = bt->hvec->seg[i];
    g.n = pr->nodes(pr->finest());
    g.bps = (int)std::min(1024L, std::max(1L, (g.n + 4095) / 4096));
    g.start = blocks;
    blocks += g.bps;
    g.r = pr->fr[0];
    g.rold = pr->fr[1];
    g.z = pr->fz;
    g.p = pr->fp;
    g.q = pr->fq;
  }
  bt->vec_blocks = blocks;
  if ((rc = balloc(bt, &bt->part, 2 * (size_t)blocks))) return rc;
  bt->hvec->nseg = n;
  bt->hvec->blocks = blocks;
  bt->hvec->part = bt->part;
  bt->hvec->scal = bt->scal;
  bt->hvec->active = bt->active;
  for (int i = 0; i < n; ++i) bt->hactive[i] = 1;
  PMG_HIP(hipMemcpy(bt->active, bt->hactive, (size_t)n * sizeof(int), hipMemcpyHostToDevice));
  PMG_HIP(hipMemcpy(bt->vec, bt->hvec, sizeof(BVecStage), hipMemcpyHostToDevice));
  // plans with the cached launch parameters (defaults where the cache has none)
  if (path) {
    bt->cache_path = path;
    bt->cache = read_cache(bt->cache_path);
  }
  const std::string pre = bt->arch + "/3d/";
  if (bt->p64.supported && (rc = tune(bt, bt->p64, pre + "fp64/", false, false))) return rc;
  if ((rc = tune(bt, bt->p32, pre + "fp32/", false, false))) return rc;
  if ((rc = tune(bt, bt->outer, pre + "fp64-outer/", true, false))) return rc;
  return PMG_OK;
}

template <typename T>
int stats(const Plan<T> &pl, int *n_stages, int *n_launches) {
  int groups = 0, last = -1;
  for (const Step &s : pl.steps)
    if (s.group != last) {
      ++groups;
      last = s.group;
    }
  if (n_stages) *n_stages = groups;
  if (n_launches) *n_launches = (int)pl.steps.size();
  return PMG_OK;
}

}  // namespace

extern "C" {

int pmg_batch_create(pmg_problem *const *problems, int n, const char *tuning_cache_path, pmg_batch **out) {
  if (!problems || !out) return fail(PMG_ERR_INVALID_ARG, "problems or out is NULL");
  if (n < 1 || n > PMG_BATCH_MAX) return fail(PMG_ERR_INVALID_ARG, "n must be in [1, %d], got %d", PMG_BATCH_MAX, n);
  pmg_batch *bt = nullptr;
  try {
    bt = new pmg_batch;
  } catch (const std::exception &e) {
    return fail(PMG_ERR_OUT_OF_MEMORY, "%s", e.what());
  }
  int rc;
  try {
    rc = create(bt, problems, n, tuning_cache_path);
  } catch (const std::exception &e) {
    rc = fail(PMG_ERR_OUT_OF_MEMORY, "%s", e.what());
  }
  if (rc != PMG_OK) {
    (void)hipDeviceSynchronize();
    destroy(bt);
    return rc;
  }
  *out = bt;
  return PMG_OK;
}

int pmg_batch_stats(const pmg_batch *bt, int mg_prec, int *n_stages, int *n_launches) {
  if (!bt) return fail(PMG_ERR_INVALID_ARG, "batch is NULL");
  if (int rc = check_mg((pmg_batch *)bt, mg_prec)) return rc;
  return mg_prec == PMG_FP64 ? stats(bt->p64, n_stages, n_launches) : stats(bt->p32, n_stages, n_launches);
}

int pmg_batch_vcycle(pmg_batch *bt, int mg_prec, const double *const *r, double *const *z, void *stream) {
  if (!bt) return fail(PMG_ERR_INVALID_ARG, "batch is NULL");
  if (int rc = check_mg(bt, mg_prec)) return rc;
  if (!r || !z) return fail(PMG_ERR_INVALID_ARG, "r or z is NULL");
  for (int i = 0; i < bt->n; ++i)
    if (!r[i] || !z[i]) return fail(PMG_ERR_INVALID_ARG, "r[%d] or z[%d] is NULL", i, i);
  hipStream_t s = (hipStream_t)stream;
  int rc = mg_prec == PMG_FP64 ? ready(bt, bt->p64, "fp64", false) : ready(bt, bt->p32, "fp32", false);
  if (rc || (rc = mg_prec == PMG_FP64 ? ensure_graphs(bt, bt->p64) : ensure_graphs(bt, bt->p32))) return rc;
  for (int i = 0; i < bt->n; ++i) bt->hactive[i] = 1;
  PMG_HIP(hipMemcpyAsync(bt->active, bt->hactive, (size_t)bt->n * sizeof(int), hipMemcpyHostToDevice, s));
  for (int i = 0; i < bt->n; ++i) {
    pmg_problem *pr = bt->pr[i];
    PMG_HIP(hipMemcpyAsync(pr->fr[0], r[i], (size_t)pr->nodes(pr->finest()) * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  PMG_HIP(hipGraphLaunch(mg_prec == PMG_FP64 ? bt->p64.vgraph : bt->p32.vgraph, s));
  for (int i = 0; i < bt->n; ++i) {
    pmg_problem *pr = bt->pr[i];
    PMG_HIP(hipMemcpyAsync(z[i], pr->fz, (size_t)pr->nodes(pr->finest()) * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  return PMG_OK;
}

int pmg_batch_solve(pmg_batch *bt, int mg_prec, const double *const *b, double *const *x, pmg_solve_info *infos,
                    void *stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!bt) return fail(PMG_ERR_INVALID_ARG, "batch is NULL");
  if (int rc = check_mg(bt, mg_prec)) return rc;
  if (!b || !x) return fail(PMG_ERR_INVALID_ARG, "b or x is NULL");
  for (int i = 0; i < bt->n; ++i)
    if (!b[i] || !x[i]) return fail(PMG_ERR_INVALID_ARG, "b[%d] or x[%d] is NULL", i, i);
  hipStream_t s = (hipStream_t)stream;
  int rc = mg_prec == PMG_FP64 ? ready(bt, bt->p64, "fp64", false) : ready(bt, bt->p32, "fp32", false);
  if (rc || (rc = ready(bt, bt->outer, "fp64-outer", true))) return rc;
  if ((rc = mg_prec == PMG_FP64 ? ensure_graphs(bt, bt->p64) : ensure_graphs(bt, bt->p32))) return rc;
  hipGraphExec_t g = mg_prec == PMG_FP64 ? bt->p64.igraph : bt->p32.igraph;
  const int n = bt->n;
  // x = 0, r = rold = b, p = 0; rz = 1 so that the first beta is (z,r) - (z,r) = 0
  for (int i = 0; i < n; ++i) {
    pmg_problem *pr = bt->pr[i];
    const size_t bytes = (size_t)pr->nodes(pr->finest()) * sizeof(double);
    bt->hvec->seg[i].x = x[i];
    PMG_HIP(hipMemsetAsync(x[i], 0, bytes, s));
    PMG_HIP(hipMemcpyAsync(pr->fr[0], b[i], bytes, hipMemcpyDeviceToDevice, s));
    PMG_HIP(hipMemcpyAsync(pr->fr[1], b[i], bytes, hipMemcpyDeviceToDevice, s));
    PMG_HIP(hipMemsetAsync(pr->fp, 0, bytes, s));
  }
  PMG_HIP(hipMemcpyAsync(bt->vec, bt->hvec, sizeof(BVecStage), hipMemcpyHostToDevice, s));
  std::memset(bt->hscal, 0, (size_t)n * S_COUNT * sizeof(double));
  for (int i = 0; i < n; ++i) {
    bt->hscal[i * S_COUNT + S_RZ] = 1.0;
    bt->hactive[i] = 1;
  }
  PMG_HIP(hipMemcpyAsync(bt->scal, bt->hscal, (size_t)n * S_COUNT * sizeof(double), hipMemcpyHostToDevice, s));
  PMG_HIP(hipMemcpyAsync(bt->active, bt->hactive, (size_t)n * sizeof(int), hipMemcpyHostToDevice, s));
  if ((rc = vec_op(bt, 4, s))) return rc;
  PMG_HIP(hipMemcpyAsync(bt->hscal, bt->scal, (size_t)n * S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
  PMG_HIP(hipStreamSynchronize(s));
  std::vector<double> nb(n), rel(n, 0.0);
  std::vector<int> its(n, 0), status(n, PMG_OK);
  int max_it = 0, live = 0;
  for (int i = 0; i < n; ++i) {
    nb[i] = std::sqrt(bt->hscal[i * S_COUNT + S_BB]);
    rel[i] = nb[i] == 0.0 ? 0.0 : std::sqrt(bt->hscal[i * S_COUNT + S_RR]) / nb[i];
    bt->hactive[i] = rel[i] > bt->pr[i]->cfg.rtol ? 1 : 0;
    live += bt->hactive[i];
    max_it = std::max(max_it, bt->pr[i]->cfg.max_iter);
  }
  for (int it = 1; it <= max_it && live > 0; ++it) {
    PMG_HIP(hipMemcpyAsync(bt->active, bt->hactive, (size_t)n * sizeof(int), hipMemcpyHostToDevice, s));
    PMG_HIP(hipGraphLaunch(g, s));
    PMG_HIP(hipMemcpyAsync(bt->hscal, bt->scal, (size_t)n * S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    PMG_HIP(hipStreamSynchronize(s));
    live = 0;
    for (int i = 0; i < n; ++i) {
      if (!bt->hactive[i]) continue;
      const double pq = bt->hscal[i * S_COUNT + S_PQ];
      rel[i] = std::sqrt(bt->hscal[i * S_COUNT + S_RR]) / nb[i];
      its[i] = it;
      if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(rel[i])) {
        status[i] = PMG_ERR_BREAKDOWN;
        bt->hactive[i] = 0;
      } else if (rel[i] <= bt->pr[i]->cfg.rtol) {
        bt->hactive[i] = 0;
      } else if (it >= bt->pr[i]->cfg.max_iter) {
        status[i] = PMG_ERR_NOT_CONVERGED;
        bt->hactive[i] = 0;
      }
      live += bt->hactive[i];
    }
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int ret = PMG_OK;
  for (int i = 0; i < n; ++i) {
    if (infos) {
      infos[i].iterations = its[i];
      infos[i].rel_residual = rel[i];
      infos[i].seconds = secs;
      infos[i].status = status[i];
    }
    if (status[i] != PMG_OK && ret == PMG_OK) {
      ret = status[i];
      fail(ret, "problem %d: %s after %d iterations (relative residual %g)", i,
           ret == PMG_ERR_BREAKDOWN ? "flexible CG breakdown" : "no convergence", its[i], rel[i]);
    }
  }
  return ret;
}

void pmg_destroy_batch(pmg_batch *bt) {
  if (!bt) return;
  (void)hipDeviceSynchronize();
  destroy(bt);
}

}  // extern "C"
