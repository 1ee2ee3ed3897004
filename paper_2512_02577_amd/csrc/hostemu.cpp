// CPU emulation of the kernel bodies (validation build, not part of libpmg.so).
//
// Runs the same templated bodies the HIP kernels run, one workgroup at a time with a
// single thread (NT = 1) and an exactly sized heap arena in place of LDS, so that index
// arithmetic, LDS layouts and tables can be checked against the oracle and under a
// bounds checker on a machine without a GPU.  Only the test suite loads it.
#include <cstdio>
#include <cstring>
#include <vector>

#include "dispatch.h"
#include "host_tables.h"

using namespace pmg;

namespace {

struct HostTabs {
  Tables t;
  DevTabs<double> d{};
  void bind() {
    std::memset(&d, 0, sizeof(d));
    for (size_t l = 0; l < t.lev.size(); ++l) {
      d.Kp[l] = t.lev[l].Kp.data();
      d.Mp[l] = t.lev[l].Mp.data();
      d.invD[l] = t.lev[l].invD.data();
      d.Tp[l] = t.lev[l].Tp.empty() ? nullptr : t.lev[l].Tp.data();
      d.TpT[l] = t.lev[l].TpT.empty() ? nullptr : t.lev[l].TpT.data();
    }
    d.Kr = t.Kr.data();
    d.Mr = t.Mr.data();
    d.Kt = t.Kt.data();
    d.Mt = t.Mt.data();
    d.W1 = t.W1.data();
    d.Wr = t.Wr.data();
  }
};

bool make_tabs(HostTabs &h, int dim, int p, const int *deg, int L, const double *omega, int n_coarse) {
  std::vector<int> degrees(deg, deg + L);
  dvec om;
  if (omega) om.assign(omega, omega + L);
  build_tables(dim, p, degrees, om, n_coarse, h.t);
  h.bind();
  return true;
}

double cscale(int dim, int n) { return dim == 3 ? 1.0 / n : 1.0; }

template <int DIM>
struct EmuSmooth {
  template <int P, class H>
  struct F {
    static int run(const SmoothArgs<double> &base, int n, int color_dir, bool local_only, int n_blocks) {
      using B = PatchBody<DIM, double, 1, P, H>;
      std::vector<double> lds(B::size);
      if (local_only) {
        for (int blk = 0; blk < n_blocks; ++blk) B::local_only(0, blk, lds.data(), base);
        return 0;
      }
      const int ncol = 1 << DIM;
      for (int ci = 0; ci < ncol; ++ci) {
        const int col = color_dir > 0 ? ci : ncol - 1 - ci;
        SmoothArgs<double> a = base;
        a.n_patch = 1;
        for (int d = 0; d < 3; ++d) {
          if (d >= DIM) {
            a.first[d] = 0;
            a.cnt[d] = 1;
            continue;
          }
          const int bit = (col >> d) & 1;
          a.first[d] = bit ? 1 : 2;
          a.cnt[d] = a.first[d] <= n - 1 ? (n - 1 - a.first[d]) / 2 + 1 : 0;
          a.n_patch *= a.cnt[d];
        }
        for (int blk = 0; blk < a.n_patch; ++blk) B::smooth_patch(0, blk, lds.data(), a);
      }
      return 0;
    }
  };
};

template <int DIM, bool RESID>
struct EmuApply {
  template <int P>
  struct F {
    static int run(ApplyArgs<double> a) {
      constexpr int TC = tile_cells(P);
      using B = ApplyBody<DIM, double, 1, P, TC, RESID>;
      std::vector<double> lds(B::size);
      a.ntile = (a.n + TC - 1) / TC;
      a.n_tiles = DIM == 3 ? a.ntile * a.ntile * a.ntile : a.ntile * a.ntile;
      for (int blk = 0; blk < a.n_tiles; ++blk) B::run(0, blk, lds.data(), a);
      return 0;
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

}  // namespace

extern "C" {

// One smoother application (all colors) on a single Cartesian level of n^dim cells.
int pmgemu_smooth(int dim, int n, int p, const int *deg, int L, const double *omega, int full, int n_iter,
                  int color_dir, double *u, const double *b) {
  HostTabs h;
  make_tabs(h, dim, p, deg, L, omega, n);
  SmoothArgs<double> a{};
  a.tb = h.d;
  a.c = cscale(dim, n);
  a.cinv = 1.0 / a.c;
  a.n = n;
  a.full = full;
  a.n_iter = n_iter;
  a.u = u;
  a.b = b;
  const int code = hierarchy_code(p, deg, L);
  if (code < 0) return -2;
  if (dim == 3) return dispatch_hierarchy<EmuSmooth<3>::F>(p, code, a, n, color_dir, false, 0);
  return dispatch_hierarchy<EmuSmooth<2>::F>(p, code, a, n, color_dir, false, 0);
}

int pmgemu_local_solve(int dim, int n, int p, const int *deg, int L, const double *omega, int full, int n_iter,
                       int n_blocks, const double *r, double *d) {
  HostTabs h;
  make_tabs(h, dim, p, deg, L, omega, n);
  SmoothArgs<double> a{};
  a.tb = h.d;
  a.c = cscale(dim, n);
  a.cinv = 1.0 / a.c;
  a.n = n;
  a.full = full;
  a.n_iter = n_iter;
  a.r_blocks = r;
  a.d_blocks = d;
  const int code = hierarchy_code(p, deg, L);
  if (code < 0) return -2;
  if (dim == 3) return dispatch_hierarchy<EmuSmooth<3>::F>(p, code, a, n, 1, true, n_blocks);
  return dispatch_hierarchy<EmuSmooth<2>::F>(p, code, a, n, 1, true, n_blocks);
}

int pmgemu_apply(int dim, int n, int p, int resid, const double *u, const double *b, double *out) {
  Tables t;
  build_tables(dim, p, std::vector<int>{p}, {}, n, t);
  ApplyArgs<double> a{};
  a.Kt = t.Kt.data();
  a.Mt = t.Mt.data();
  a.c = cscale(dim, n);
  a.n = n;
  a.u = u;
  a.b = b;
  a.out = out;
  if (dim == 3)
    return resid ? dispatch_degree<EmuApply<3, true>::F>(p, a) : dispatch_degree<EmuApply<3, false>::F>(p, a);
  return resid ? dispatch_degree<EmuApply<2, true>::F>(p, a) : dispatch_degree<EmuApply<2, false>::F>(p, a);
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

int pmgemu_coarse_solve(int dim, int n0, int p, const double *r, double *z) {
  Tables t;
  build_tables(dim, p, std::vector<int>{p}, {}, n0, t);
  const int m = t.m0;
  std::vector<double> w1((size_t)(dim == 3 ? m * m * m : m * m)), w2(w1.size());
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
  if (dim == 3)
    CoarseBody<3, double, 1>::run(0, a);
  else
    CoarseBody<2, double, 1>::run(0, a);
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
