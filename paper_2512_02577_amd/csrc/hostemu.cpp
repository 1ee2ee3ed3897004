// CPU emulation of the kernel bodies (validation build, not part of libpmg.so).
//
// Runs the same templated bodies the HIP kernels run, one workgroup at a time, with an
// exactly sized heap arena in place of LDS, so that index arithmetic, LDS layouts, tables
// and the workgroup's barriers can be checked against the oracle and under AddressSanitizer
// / ThreadSanitizer on a machine without a GPU.  A workgroup runs either on one thread
// (NT = 1: every lane loop sequential) or on a team of NT host threads, one per lane, with
// a barrier for every workgroup barrier of the body: this executes the lane-count dependent
// paths (split stages, strided per-lane reads, read-ahead registers) exactly as the device
// launches them.  Only the test suite loads it.
//
// Lane codes of the entry points: 0 = one lane; 1 = the lane count of the library's
// launch of that body (patch_threads, apply_threads, ...); 2 = 256 lanes (the latency
// variant of the patch smoother); 3 = half the library's count (the patch smoother's kernel
// of large launches at 3D degrees 4 and 5).  Table modes: 0 = every 1D table in its own exactly sized
// vector; 1 = the library's concatenated table block (tab_layout.h).
#include <pthread.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "bodies_metric.h"
#include "constants.h"
#include "dispatch.h"
#include "geometry.h"
#include "hex_setup.h"
#include "host_tables.h"
#include "tab_layout.h"

using namespace pmg;

namespace {

// NT host threads standing in for the lanes of one workgroup.
class Team final : public HostTeam {
 public:
  explicit Team(int nt) : nt_(nt), slot_(nt, 0.0) { pthread_barrier_init(&bar_, nullptr, (unsigned)nt); }
  ~Team() override { pthread_barrier_destroy(&bar_); }
  void sync() override { pthread_barrier_wait(&bar_); }
  double sum(int tid, double v) override {
    slot_[tid] = v;
    sync();
    double s = 0.0;
    for (double x : slot_) s += x;
    sync();
    return s;
  }
  template <class F>
  void run(const F &f) {
    std::vector<std::thread> th;
    th.reserve(nt_);
    for (int t = 0; t < nt_; ++t)
      th.emplace_back([this, &f, t] {
        host_team = this;
        f(t);
        host_team = nullptr;
      });
    for (auto &x : th) x.join();
  }

 private:
  int nt_;
  std::vector<double> slot_;
  pthread_barrier_t bar_;
};

// Runs f(tid) for the NT lanes of a workgroup.
template <int NT, class F>
void run_lanes(const F &f) {
  if constexpr (NT == 1) {
    f(0);
  } else {
    Team t(NT);
    t.run(f);
  }
}

// A launch of nblk workgroups on one arena (the workgroups run one after the other, with a
// barrier between them, as the global-arena kernels loop).
template <int NT, class F>
void launch(int nblk, std::vector<double> &arena, const F &body) {
  run_lanes<NT>([&](int tid) {
    for (int blk = 0; blk < nblk; ++blk) {
      body(tid, blk, arena.data());
      PMG_SYNC();
    }
  });
}

struct HostTabs {
  Tables t;
  DevTabs<double> d{};
  std::vector<double> flat;  // table mode 1: the library's block
  void bind(int mode) {
    std::memset(&d, 0, sizeof(d));
    if (mode == 1) {
      std::vector<size_t> off;
      flat.clear();
      flatten_tabs(t, flat, off);
      bind_tabs(d, t, flat.data(), off);
      return;
    }
    for (size_t l = 0; l < t.lev.size(); ++l) {
      d.Kp[l] = t.lev[l].Kp.data();
      d.Mp[l] = t.lev[l].Mp.data();
      d.invD[l] = t.lev[l].invD.data();
      d.Tp[l] = t.lev[l].Tp.empty() ? nullptr : t.lev[l].Tp.data();
      d.TpT[l] = t.lev[l].TpT.empty() ? nullptr : t.lev[l].TpT.data();
      d.S[l] = t.lev[l].S.empty() ? nullptr : t.lev[l].S.data();
      d.ST[l] = t.lev[l].ST.empty() ? nullptr : t.lev[l].ST.data();
      d.Linv[l] = t.lev[l].Linv.empty() ? nullptr : t.lev[l].Linv.data();
    }
    d.Kr = t.Kr.data();
    d.Mr = t.Mr.data();
    d.Kt = t.Kt.data();
    d.Mt = t.Mt.data();
    d.W1 = t.W1.data();
    d.Wr = t.Wr.data();
  }
};

void make_tabs(HostTabs &h, int dim, int p, const int *deg, int L, const double *omega, int n_coarse, int mode) {
  std::vector<int> degrees(deg, deg + L);
  dvec om;
  if (omega) om.assign(omega, omega + L);
  build_tables(dim, p, degrees, om, n_coarse, h.t);
  h.bind(mode);
}

double cscale(int dim, int n) { return dim == 3 ? 1.0 / n : 1.0; }

// first vertex coordinate and patch count per axis of color col (the library's do_smooth)
template <typename A>
void color_range(int dim, int n, int col, A &a, int first_odd, int first_even) {
  a.n_patch = 1;
  for (int d = 0; d < 3; ++d) {
    if (d >= dim) {
      a.first[d] = 0;
      a.cnt[d] = 1;
      continue;
    }
    a.first[d] = (col >> d) & 1 ? first_odd : first_even;
    a.cnt[d] = a.first[d] <= n - 1 ? (n - 1 - a.first[d]) / 2 + 1 : 0;
    a.n_patch *= a.cnt[d];
  }
}

template <int DIM>
struct EmuSmooth {
  template <int P, class H>
  struct F {
    template <int NT, bool ONE>
    static int go(const SmoothArgs<double> &base, int n, int color_dir, bool local_only, int n_blocks) {
      using B = PatchBody<DIM, double, NT, P, H>;
      // exactly what the device launch gets
      std::vector<double> lds(ONE && !local_only ? B::arena_one() : B::arena(base.n_iter));
      if (local_only) {
        launch<NT>(n_blocks, lds, [&](int tid, int blk, double *ar) { B::local_only(tid, blk, ar, base); });
        return 0;
      }
      const int ncol = 1 << DIM;
      for (int ci = 0; ci < ncol; ++ci) {
        const int col = color_dir > 0 ? ci : ncol - 1 - ci;
        SmoothArgs<double> a = base;
        color_range(DIM, n, col, a, 1, 2);
        if (a.n_patch == 0) continue;
        launch<NT>(a.n_patch, lds,
                   [&](int tid, int blk, double *ar) { B::template smooth_patch<ONE>(tid, blk, ar, a); });
      }
      return 0;
    }
    static int run(const SmoothArgs<double> &base, int n, int color_dir, bool local_only, int n_blocks, int lanes,
                   int one) {
      const bool o = one != 0;
      if (o && (base.full || base.n_iter != 1 || base.direct || base.reinf))
        return -3;  // ONE compiles the default solver only
      switch (lanes) {
        case 0: return o ? go<1, true>(base, n, color_dir, local_only, n_blocks)
                         : go<1, false>(base, n, color_dir, local_only, n_blocks);
        case 1: return o ? go<patch_threads(P, DIM), true>(base, n, color_dir, local_only, n_blocks)
                         : go<patch_threads(P, DIM), false>(base, n, color_dir, local_only, n_blocks);
        case 2: return o ? go<256, true>(base, n, color_dir, local_only, n_blocks)
                         : go<256, false>(base, n, color_dir, local_only, n_blocks);
        case 3:
          if constexpr (DIM == 3 && (P == 4 || P == 5))
            return o ? go<patch_threads(P, DIM) / 2, true>(base, n, color_dir, local_only, n_blocks)
                     : go<patch_threads(P, DIM) / 2, false>(base, n, color_dir, local_only, n_blocks);
          else
            return -1;
        default: return -1;
      }
    }
  };
};

// kind: 0 v = A u, 1 v = b - A u, 2 v = M u (mass).  3D degrees with a marching apply run
// that body (as the library does); zsplit 0 takes the library's z segments, 1 one segment
// per xy tile (every layer of the mesh in one workgroup).
template <int DIM, int KIND>
struct EmuApply {
  static constexpr bool RESID = KIND == 1, MASS = KIND == 2;
  template <int P>
  struct F {
    template <int NT>
    static int go(ApplyArgs<double> a, int zsplit) {
      if constexpr (DIM == 3 && march_tile(P) > 0) {
        using B = MarchBody<double, NT, P, march_tile(P), march_tile_y(P), march_group(P), P * (tile_cells(P) + 1) + 1,
                            RESID, MASS>;
        std::vector<double> lds(B::size);
        int nseg;
        march_geometry(a.n, march_tile(P), march_tile_y(P), zsplit ? 1 : kMarchBlocks, a.mt, a.mty, nseg, a.zc);
        a.n_tiles = a.mt * a.mty * nseg;
        launch<NT>(a.n_tiles, lds, [&](int tid, int blk, double *ar) { B::run(tid, blk, ar, a); });
        return 0;
      } else {
        constexpr int TC = tile_cells(P);
        using B = ApplyBody<DIM, double, NT, P, TC, RESID, MASS>;
        std::vector<double> lds(B::size);
        a.ntile = (a.n + TC - 1) / TC;
        a.n_tiles = DIM == 3 ? a.ntile * a.ntile * a.ntile : a.ntile * a.ntile;
        launch<NT>(a.n_tiles, lds, [&](int tid, int blk, double *ar) { B::run(tid, blk, ar, a); });
        return 0;
      }
    }
    static int run(const ApplyArgs<double> &a, int lanes, int zsplit) {
      if (lanes == 0) return go<1>(a, zsplit);
      constexpr int NT = (DIM == 3 && march_tile(P) > 0) ? march_threads(P) : apply_threads(P);
      if (lanes == 1) return go<NT>(a, zsplit);
      return -1;
    }
  };
};

template <int DIM, bool RESTRICT>
struct EmuTransfer {
  template <int P>
  struct F {
    static int run(const TransferArgs<double> &a) {
      PassArgs<double> pa[3];
      const int np = transfer_passes<double>(DIM, P, RESTRICT, a, pa);
      for (int k = 0; k < np; ++k) {
        const long total = (long)pa[k].oe[0] * pa[k].oe[1] * pa[k].oe[2];
        for (long g = 0; g < total; ++g) {
          if (RESTRICT)
            TransferPass<double, P, true, false>::node(g, pa[k]);
          else if (k == np - 1)
            TransferPass<double, P, false, true>::node(g, pa[k]);
          else
            TransferPass<double, P, false, false>::node(g, pa[k]);
        }
      }
      return 0;
    }
  };
};

// ---- general path ----
struct HostQ {
  QTab t;
  QTabDev<double> d{};
  void bind() {
    d.B = t.B.data(); d.BT = t.BT.data(); d.Dq = t.Dq.data(); d.DqT = t.DqT.data();
    d.Bpc = t.Bpc.data(); d.Bpi = t.Bpi.data(); d.BpiT = t.BpiT.data(); d.Dqp = t.Dqp.data(); d.DqpT = t.DqpT.data();
  }
};

template <int DIM>
struct EmuMetricApply {
  template <int P>
  struct F {
    template <int NT>
    static int go(const MetricApplyArgs<double, double> &base) {
      using B = MetricApplyBody<DIM, double, double, NT, P>;
      std::vector<double> lds(B::size);
      const int ncol = 1 << DIM, n = base.n;
      for (int col = 0; col < ncol; ++col) {
        MetricApplyArgs<double, double> a = base;
        a.n_cells = 1;
        for (int d = 0; d < 3; ++d) {
          if (d >= DIM) { a.first[d] = 0; a.cnt[d] = 1; continue; }
          a.first[d] = (col >> d) & 1;
          a.cnt[d] = a.first[d] <= n - 1 ? (n - 1 - a.first[d]) / 2 + 1 : 0;
          a.n_cells *= a.cnt[d];
        }
        if (a.n_cells == 0) continue;
        launch<NT>(a.n_cells, lds, [&](int tid, int blk, double *ar) { B::run(tid, blk, ar, a); });
      }
      return 0;
    }
    static int run(const MetricApplyArgs<double, double> &base, int lanes) {
      if (lanes == 0) return go<1>(base);
      if (lanes == 1) return go<metric_apply_threads(P)>(base);
      return -1;
    }
  };
};

template <int DIM>
struct EmuMetricSmooth {
  template <int P, class H>
  struct F {
    template <int NT, bool ONE>
    static int go(const MetricSmoothArgs<double, double> &base, int n, int color_dir, bool local_only, int nb) {
      using B = MetricPatchBody<DIM, double, double, NT, P, H>;
      std::vector<double> lds(B::arena(base.n_iter));  // exactly what the device launch gets
      if (local_only) {
        launch<NT>(nb, lds, [&](int tid, int blk, double *ar) { B::local_only(tid, blk, ar, base); });
        return 0;
      }
      const int ncol = 1 << DIM;
      for (int ci = 0; ci < ncol; ++ci) {
        const int col = color_dir > 0 ? ci : ncol - 1 - ci;
        MetricSmoothArgs<double, double> a = base;
        color_range(DIM, n, col, a, 1, 2);
        if (a.n_patch == 0) continue;
        launch<NT>(a.n_patch, lds,
                   [&](int tid, int blk, double *ar) { B::template smooth_patch<ONE>(tid, blk, ar, a); });
      }
      return 0;
    }
    static int run(const MetricSmoothArgs<double, double> &base, int n, int color_dir, bool local_only, int nb,
                   int lanes, int one) {
      const bool o = one != 0;
      if (o && (base.full || base.n_iter != 1)) return -3;
      constexpr int W = metric_patch_threads(P, sizeof(double));
      if (lanes == 0) return o ? go<1, true>(base, n, color_dir, local_only, nb)
                               : go<1, false>(base, n, color_dir, local_only, nb);
      if (lanes == 1) return o ? go<W, true>(base, n, color_dir, local_only, nb)
                               : go<W, false>(base, n, color_dir, local_only, nb);
      return -1;
    }
  };
};

// per-patch inverse diagonals of one p-level from the metric (host loops over the bodies)
template <int DIM>
void emu_inv_diag(int n, int q, double omega, const dvec &G, dvec &invD) {
  const QTab t = make_qtab(q);
  const int k = q + 1;
  dvec Dn((size_t)t.nq * k, 0.0);
  for (int g = 0; g < t.nq; ++g)
    for (int a = 0; a < k; ++a) {
      double s = 0.0;
      for (int h = 0; h < t.nq; ++h) s += t.Dq[(size_t)g * t.nq + h] * t.B[(size_t)h * k + a];
      Dn[(size_t)g * k + a] = s;
    }
  const long ncell = DIM == 3 ? (long)n * n * n : (long)n * n, kd = DIM == 3 ? k * k * k : k * k;
  dvec cd((size_t)(ncell * kd));
  for (long tt = 0; tt < ncell * kd; ++tt) cell_diag<DIM, double>(tt, q, t.B.data(), Dn.data(), G.data(), cd.data());
  const long e1 = 2 * q - 1, nd = DIM == 3 ? e1 * e1 * e1 : e1 * e1, np = DIM == 3 ? (long)(n - 1) * (n - 1) * (n - 1)
                                                                                       : (long)(n - 1) * (n - 1);
  invD.assign((size_t)(np * nd), 0.0);
  for (long tt = 0; tt < np * nd; ++tt) patch_inv_diag<DIM, double>(tt, q, n, omega, cd.data(), invD.data());
}

// General hex meshes: the stored-map bodies over the colors of a HexHost
template <int DIM>
struct EmuHexSmooth {
  template <int P, class H>
  struct F {
    template <int NT, bool ONE>
    static int go(const MetricSmoothArgs<double, double> &base, const HexHost &h, int color_dir) {
      using B = MetricPatchBody<DIM, double, double, NT, P, H>;
      std::vector<double> lds(B::arena(base.n_iter));
      const int ncol = (int)h.pfirst.size() - 1;
      for (int ci = 0; ci < ncol; ++ci) {
        const int col = color_dir > 0 ? ci : ncol - 1 - ci;
        MetricSmoothArgs<double, double> a = base;
        a.plist = h.plist.data() + h.pfirst[col];
        a.n_patch = h.pfirst[col + 1] - h.pfirst[col];
        launch<NT>(a.n_patch, lds,
                   [&](int tid, int blk, double *ar) { B::template smooth_patch_stored<ONE>(tid, blk, ar, a); });
      }
      return 0;
    }
    static int run(const MetricSmoothArgs<double, double> &base, const HexHost &h, int color_dir, int lanes, int one) {
      const bool o = one != 0;
      if (o && (base.full || base.n_iter != 1)) return -3;
      constexpr int W = metric_patch_threads(P, sizeof(double));
      if (lanes == 0) return o ? go<1, true>(base, h, color_dir) : go<1, false>(base, h, color_dir);
      if (lanes == 1) return o ? go<W, true>(base, h, color_dir) : go<W, false>(base, h, color_dir);
      return -1;
    }
  };
};

template <int DIM>
struct EmuHexApply {
  template <int P>
  struct F {
    template <int NT>
    static int go(const MetricApplyArgs<double, double> &base, const HexHost &h) {
      using B = MetricApplyBody<DIM, double, double, NT, P>;
      std::vector<double> lds(B::size);
      const int ncol = (int)h.cfirst.size() - 1;
      for (int col = 0; col < ncol; ++col) {
        MetricApplyArgs<double, double> a = base;
        a.clist = h.clist.data() + h.cfirst[col];
        a.n_cells = h.cfirst[col + 1] - h.cfirst[col];
        launch<NT>(a.n_cells, lds, [&](int tid, int blk, double *ar) { B::template run<true>(tid, blk, ar, a); });
      }
      return 0;
    }
    static int run(const MetricApplyArgs<double, double> &base, const HexHost &h, int lanes) {
      if (lanes == 0) return go<1>(base, h);
      if (lanes == 1) return go<metric_apply_threads(P)>(base, h);
      return -1;
    }
  };
};

// metric of degree q on the cells of a HexHost (corners in the common frame)
bool hex_metric(const HexHost &h, int q, dvec &G) {
  const int dim = h.dim, ncn = 1 << dim;
  return metric_cells(
      dim, h.n_cells,
      [&](long c, double X[8][3]) {
        for (int j = 0; j < ncn; ++j)
          for (int a = 0; a < dim; ++a) X[j][a] = h.xyz[(size_t)h.cverts[(size_t)c * ncn + j] * dim + a];
      },
      q, nullptr, G);
}

// per-patch inverse diagonals of one p-level on a HexHost
template <int DIM>
void emu_hex_inv_diag(const HexHost &h, int q, double omega, const dvec &G, dvec &invD) {
  const QTab t = make_qtab(q);
  const int k = q + 1;
  dvec Dn((size_t)t.nq * k, 0.0);
  for (int g = 0; g < t.nq; ++g)
    for (int a = 0; a < k; ++a) {
      double s = 0.0;
      for (int hh = 0; hh < t.nq; ++hh) s += t.Dq[(size_t)g * t.nq + hh] * t.B[(size_t)hh * k + a];
      Dn[(size_t)g * k + a] = s;
    }
  const long kd = DIM == 3 ? k * k * k : k * k;
  dvec cd((size_t)(h.n_cells * kd));
  for (long tt = 0; tt < h.n_cells * kd; ++tt) cell_diag<DIM, double>(tt, q, t.B.data(), Dn.data(), G.data(), cd.data());
  const long e1 = 2 * q - 1, nd = DIM == 3 ? e1 * e1 * e1 : e1 * e1, np = (long)h.pvert.size();
  invD.assign((size_t)(np * nd), 0.0);
  for (long tt = 0; tt < np * nd; ++tt)
    patch_inv_diag_list<DIM, double>(tt, q, h.pcells.data(), omega, cd.data(), invD.data());
}

// Cartesian patch-solver arguments: local 0 half V-cycle, 1 full V-cycle, 2 exact solve;
// reinf: Cartesian-reinforced p-level preconditioner (damping omega) instead of Jacobi
void set_local(SmoothArgs<double> &a, const HostTabs &h, int local, int reinf) {
  a.full = local == 1;
  a.direct = local == 2;
  a.reinf = reinf;
  for (size_t l = 0; l < h.t.lev.size() && l < 4; ++l) a.om.w[l] = h.t.omega[l];
}

}  // namespace

extern "C" {

// Metric-path apply (resid: out = b - A u) on one level; verts: (n+1)^d x d or NULL for
// the Cartesian box; coef: per Gauss point of degree p, or NULL.
int pmgemu_metric_apply(int dim, int n, int p, const double *verts, const double *coef, int resid, const double *u,
                        const double *b, double *out, int lanes) {
  dvec V = verts ? dvec(verts, verts + (size_t)(dim == 3 ? (n + 1) * (n + 1) * (n + 1) : (n + 1) * (n + 1)) * dim)
                 : cartesian_vertices(dim, n);
  dvec G;
  if (!metric(dim, n, V, p, coef, G)) return -1;
  HostQ hq;
  hq.t = make_qtab(p);
  hq.bind();
  const long m = (long)p * n + 1, N = dim == 3 ? m * m * m : m * m;
  for (long g = 0; g < N; ++g) metric_apply_init<double>(g, dim, (int)m, resid != 0, b, u, out);
  MetricApplyArgs<double, double> a{};
  a.qt = hq.d;
  a.G = G.data();
  a.n = n;
  a.sign = resid ? -1.0 : 1.0;
  a.u = u;
  a.out = out;
  if (dim == 3) return dispatch_degree<EmuMetricApply<3>::F>(p, a, lanes);
  return dispatch_degree<EmuMetricApply<2>::F>(p, a, lanes);
}

// Metric-path smoother (all colors) or local solve (nb > 0: r/d blocks) on one level.
// coefs: L pointers (Gauss-point coefficient per p-level, NULL entries for mu = 1).
int pmgemu_metric_smooth(int dim, int n, int p, const int *deg, int L, const double *omega, int full, int n_iter,
                         int color_dir, const double *verts, const double *const *coefs, double *u, const double *b,
                         int nb, const double *r, double *d, int lanes, int one) {
  dvec V = verts ? dvec(verts, verts + (size_t)(dim == 3 ? (n + 1) * (n + 1) * (n + 1) : (n + 1) * (n + 1)) * dim)
                 : cartesian_vertices(dim, n);
  Tables tab;
  std::vector<int> degrees(deg, deg + L);
  build_tables(dim, p, degrees, dvec(omega, omega + L), n, tab);
  std::vector<HostQ> hq(L);
  std::vector<dvec> G(L), invD(L);
  MetricSmoothArgs<double, double> a{};
  for (int l = 0; l < L; ++l) {
    hq[l].t = make_qtab(deg[l]);
    hq[l].bind();
    if (!metric(dim, n, V, deg[l], coefs ? coefs[l] : nullptr, G[l])) return -1;
    if (dim == 3)
      emu_inv_diag<3>(n, deg[l], l == 0 ? 1.0 : omega[l], G[l], invD[l]);
    else
      emu_inv_diag<2>(n, deg[l], l == 0 ? 1.0 : omega[l], G[l], invD[l]);
    a.lev[l].qt = hq[l].d;
    a.lev[l].G = G[l].data();
    a.lev[l].invD = invD[l].data();
    a.lev[l].Tp = tab.lev[l].Tp.empty() ? nullptr : tab.lev[l].Tp.data();
    a.lev[l].TpT = tab.lev[l].TpT.empty() ? nullptr : tab.lev[l].TpT.data();
  }
  a.n = n;
  a.full = full;
  a.n_iter = n_iter;
  a.u = u;
  a.b = b;
  a.r_blocks = r;
  a.d_blocks = d;
  const int code = hierarchy_code(p, deg, L);
  if (code < 0) return -2;
  if (dim == 3) return dispatch_hierarchy<EmuMetricSmooth<3>::F>(p, code, a, n, color_dir, nb > 0, nb, lanes, one);
  return dispatch_hierarchy<EmuMetricSmooth<2>::F>(p, code, a, n, color_dir, nb > 0, nb, lanes, one);
}

// General hex mesh (hex_build's arrays): the stored-map apply (resid: out = b - A u).
int pmgemu_hex_apply(int dim, int p, long nv, const double *xyz, long nc, const int32_t *cv, long ndof,
                     const int32_t *cd, int resid, const double *u, const double *b, double *out, int lanes) {
  HexHost h;
  std::string err;
  if (int rc = hex_build(dim, p, nv, xyz, nc, cv, ndof, cd, h, err)) return rc;
  dvec G;
  if (!hex_metric(h, p, G)) return -1;
  HostQ hq;
  hq.t = make_qtab(p);
  hq.bind();
  for (long g = 0; g < ndof; ++g) hex_apply_init<double>(g, resid != 0, h.bnd.data(), b, u, out);
  MetricApplyArgs<double, double> a{};
  a.qt = hq.d;
  a.G = G.data();
  a.sign = resid ? -1.0 : 1.0;
  a.u = u;
  a.out = out;
  a.cdof = h.cdofs.data();
  a.bnd = h.bnd.data();
  if (dim == 3) return dispatch_degree<EmuHexApply<3>::F>(p, a, h, lanes);
  return dispatch_degree<EmuHexApply<2>::F>(p, a, h, lanes);
}

// General hex mesh: one smoother application over the DSATUR colors (paper p-hierarchy;
// omega: one damping per p-level, coarsest first).
int pmgemu_hex_smooth(int dim, int p, const double *omega, long nv, const double *xyz, long nc, const int32_t *cv,
                      long ndof, const int32_t *cd, int full, int n_iter, int color_dir, double *u, const double *b,
                      int lanes, int one) {
  HexHost h;
  std::string err;
  if (int rc = hex_build(dim, p, nv, xyz, nc, cv, ndof, cd, h, err)) return rc;
  std::vector<int> deg;
  for (int x = 1; x < p; x = 2 * x + 1) deg.push_back(x);
  deg.push_back(p);
  const int L = (int)deg.size();
  Tables tab;
  build_tables(dim, p, deg, dvec(omega, omega + L), 2, tab);
  std::vector<HostQ> hq(L);
  std::vector<dvec> G(L), invD(L);
  MetricSmoothArgs<double, double> a{};
  for (int l = 0; l < L; ++l) {
    hq[l].t = make_qtab(deg[l]);
    hq[l].bind();
    if (!hex_metric(h, deg[l], G[l])) return -1;
    if (dim == 3)
      emu_hex_inv_diag<3>(h, deg[l], l == 0 ? 1.0 : omega[l], G[l], invD[l]);
    else
      emu_hex_inv_diag<2>(h, deg[l], l == 0 ? 1.0 : omega[l], G[l], invD[l]);
    a.lev[l].qt = hq[l].d;
    a.lev[l].G = G[l].data();
    a.lev[l].invD = invD[l].data();
    a.lev[l].Tp = tab.lev[l].Tp.empty() ? nullptr : tab.lev[l].Tp.data();
    a.lev[l].TpT = tab.lev[l].TpT.empty() ? nullptr : tab.lev[l].TpT.data();
  }
  a.full = full;
  a.n_iter = n_iter;
  a.u = u;
  a.b = b;
  a.pmap = h.pmap.data();
  a.pcells = h.pcells.data();
  if (dim == 3) return dispatch_hierarchy<EmuHexSmooth<3>::F>(p, 0, a, h, color_dir, lanes, one);
  return dispatch_hierarchy<EmuHexSmooth<2>::F>(p, 0, a, h, color_dir, lanes, one);
}

// One smoother application (all colors) on a single Cartesian level of n^dim cells.
int pmgemu_smooth(int dim, int n, int p, const int *deg, int L, const double *omega, int local, int reinf,
                  int n_iter, int color_dir, double *u, const double *b, int lanes, int one, int tabmode) {
  HostTabs h;
  make_tabs(h, dim, p, deg, L, omega, n, tabmode);
  SmoothArgs<double> a{};
  a.tb = h.d;
  a.c = cscale(dim, n);
  a.cinv = 1.0 / a.c;
  a.n = n;
  set_local(a, h, local, reinf);
  a.n_iter = n_iter;
  a.u = u;
  a.b = b;
  const int code = hierarchy_code(p, deg, L);
  if (code < 0) return -2;
  if (dim == 3) return dispatch_hierarchy<EmuSmooth<3>::F>(p, code, a, n, color_dir, false, 0, lanes, one);
  return dispatch_hierarchy<EmuSmooth<2>::F>(p, code, a, n, color_dir, false, 0, lanes, one);
}

int pmgemu_local_solve(int dim, int n, int p, const int *deg, int L, const double *omega, int local, int reinf,
                       int n_iter, int n_blocks, const double *r, double *d, int lanes, int tabmode) {
  HostTabs h;
  make_tabs(h, dim, p, deg, L, omega, n, tabmode);
  SmoothArgs<double> a{};
  a.tb = h.d;
  a.c = cscale(dim, n);
  a.cinv = 1.0 / a.c;
  a.n = n;
  set_local(a, h, local, reinf);
  a.n_iter = n_iter;
  a.r_blocks = r;
  a.d_blocks = d;
  const int code = hierarchy_code(p, deg, L);
  if (code < 0) return -2;
  if (dim == 3) return dispatch_hierarchy<EmuSmooth<3>::F>(p, code, a, n, 1, true, n_blocks, lanes, 0);
  return dispatch_hierarchy<EmuSmooth<2>::F>(p, code, a, n, 1, true, n_blocks, lanes, 0);
}

int pmgemu_apply(int dim, int n, int p, int kind, const double *u, const double *b, double *out, int lanes,
                 int zsplit) {
  Tables t;
  build_tables(dim, p, std::vector<int>{p}, {}, n, t);
  ApplyArgs<double> a{};
  a.Kt = t.Kt.data();
  a.Mt = t.Mt.data();
  a.c = kind == 2 ? 1.0 / ((dim == 3 ? (double)n : 1.0) * n * n) : cscale(dim, n);
  a.n = n;
  a.u = u;
  a.b = b;
  a.out = out;
  switch (kind + 3 * (dim == 3)) {
    case 0: return dispatch_degree<EmuApply<2, 0>::F>(p, a, lanes, zsplit);
    case 1: return dispatch_degree<EmuApply<2, 1>::F>(p, a, lanes, zsplit);
    case 2: return dispatch_degree<EmuApply<2, 2>::F>(p, a, lanes, zsplit);
    case 3: return dispatch_degree<EmuApply<3, 0>::F>(p, a, lanes, zsplit);
    case 4: return dispatch_degree<EmuApply<3, 1>::F>(p, a, lanes, zsplit);
    case 5: return dispatch_degree<EmuApply<3, 2>::F>(p, a, lanes, zsplit);
    default: return -1;
  }
}

int pmgemu_transfer(int dim, int nc, int p, int restrict_, const double *in, double *out) {
  Tables t;
  build_tables(dim, p, std::vector<int>{p}, {}, nc, t);
  TransferArgs<double> a{};
  a.W1 = t.W1.data();
  a.Wr = t.Wr.data();
  a.nc = nc;
  a.in = in;
  a.out = out;
  const long mc = (long)p * nc + 1, mf = 2L * p * nc + 1;
  std::vector<double> w1((size_t)(dim == 3 ? mc * mf * mf : mc * mf)), w2((size_t)(dim == 3 ? mf * mf * mc : 1));
  a.w1 = w1.data();
  a.w2 = w2.data();
  if (dim == 3)
    return restrict_ ? dispatch_degree<EmuTransfer<3, true>::F>(p, a) : dispatch_degree<EmuTransfer<3, false>::F>(p, a);
  return restrict_ ? dispatch_degree<EmuTransfer<2, true>::F>(p, a) : dispatch_degree<EmuTransfer<2, false>::F>(p, a);
}

// Coarse solve by fast diagonalization; lanes 0: one lane on the global work vectors,
// 1: the library's workgroup (kCoarseThreads lanes) with the work vectors in its arena.
int pmgemu_coarse_solve(int dim, int n0, int p, const double *r, double *z, int lanes) {
  Tables t;
  build_tables(dim, p, std::vector<int>{p}, {}, n0, t);
  const int m = t.m0;
  const size_t tot = dim == 3 ? (size_t)m * m * m : (size_t)m * m;
  std::vector<double> w1(tot), w2(tot), lds(2 * tot);
  CoarseArgs<double> a{};
  a.S = t.S0.data();
  a.lam = t.lam0.data();
  a.c0inv = 1.0 / cscale(dim, n0);
  a.m = m;
  a.mt = m + 2;
  a.r = r;
  a.z = z;
  a.w1 = w1.data();
  a.w2 = w2.data();
  if (lanes == 0) {
    if (dim == 3)
      CoarseBody<3, double, 1>::run(0, a);
    else
      CoarseBody<2, double, 1>::run(0, a);
    return 0;
  }
  if (lanes != 1) return -1;
  constexpr int NT = kCoarseThreads;
  run_lanes<NT>([&](int tid) {
    if (dim == 3)
      CoarseBody<3, double, NT>::run(tid, a, lds.data(), (int)lds.size());
    else
      CoarseBody<2, double, NT>::run(tid, a, lds.data(), (int)lds.size());
  });
  return 0;
}

// Tables for inspection: omega per level of the given hierarchy.
int pmgemu_omega(int dim, int p, const int *deg, int L, double *omega_out) {
  Tables t;
  build_tables(dim, p, std::vector<int>(deg, deg + L), {}, 2, t);
  for (int l = 0; l < L; ++l) omega_out[l] = t.omega[l];
  return 0;
}

}  // extern "C"
