// Bounds-checked run of every emulated kernel body (built with AddressSanitizer by
// `python -m paper_2512_02577_amd.build --asan`): each arena and vector is allocated at
// its exact size, so any out-of-range index in a body aborts the run.
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int pmgemu_smooth(int dim, int n, int p, const int *deg, int L, const double *omega, int full, int n_iter,
                  int color_dir, double *u, const double *b);
int pmgemu_local_solve(int dim, int n, int p, const int *deg, int L, const double *omega, int full, int n_iter,
                       int n_blocks, const double *r, double *d);
int pmgemu_apply(int dim, int n, int p, int resid, const double *u, const double *b, double *out);
int pmgemu_transfer(int dim, int nc, int p, int restrict_, const double *in, double *out);
int pmgemu_coarse_solve(int dim, int n0, int p, const double *r, double *z);
int pmgemu_metric_apply(int dim, int n, int p, const double *verts, const double *coef, int resid, const double *u,
                        const double *b, double *out);
int pmgemu_metric_smooth(int dim, int n, int p, const int *deg, int L, const double *omega, int full, int n_iter,
                         int color_dir, const double *verts, const double *const *coefs, double *u, const double *b,
                         int nb, const double *r, double *d);
}

static std::vector<double> rnd(size_t n, unsigned seed) {
  std::mt19937 g(seed);
  std::uniform_real_distribution<double> d(-1, 1);
  std::vector<double> v(n);
  for (auto &x : v) x = d(g);
  return v;
}

static long ipow(long b, int e) { return e ? b * ipow(b, e - 1) : 1; }

int main() {
  int fails = 0;
  for (int dim = 2; dim <= 3; ++dim)
    for (int p = 1; p <= 8; ++p)
      for (int code = 0; code < 2; ++code) {
        if (code == 1 && (p > 4 || p < 3)) continue;
        std::vector<int> deg;
        if (code == 0) {
          for (int x = 1; x < p; x = 2 * x + 1) deg.push_back(x);
          deg.push_back(p);
        } else {
          for (int x = 1; x <= p; ++x) deg.push_back(x);
        }
        std::vector<double> om(deg.size(), 0.6);
        for (int n : {2, 3, 5}) {
          if (dim == 3 && p >= 7 && n > 3) continue;
          const long N = ipow((long)p * n + 1, dim);
          auto u = rnd(N, 1), b = rnd(N, 2), out = std::vector<double>(N);
          // one Richardson step uses the smaller arena: check both sizes
          for (int it = 1; it <= 2; ++it)
            for (int full = 0; full < 2; ++full)
              fails += pmgemu_smooth(dim, n, p, deg.data(), (int)deg.size(), om.data(), full, it, 1, u.data(),
                                     b.data()) != 0;
          const long nd = ipow(2 * p - 1, dim), np = ipow(n - 1, dim);
          auto r = rnd(nd * np, 3);
          std::vector<double> d(nd * np);
          for (int it = 1; it <= 2; ++it)
            fails += pmgemu_local_solve(dim, n, p, deg.data(), (int)deg.size(), om.data(), 0, it, (int)np, r.data(),
                                        d.data()) != 0;
          if (code == 0) {
            fails += pmgemu_apply(dim, n, p, 1, u.data(), b.data(), out.data()) != 0;
            const long Nc = ipow((long)p * n + 1, dim), Nf = ipow(2L * p * n + 1, dim);
            auto fine = rnd(Nf, 4), coarse = std::vector<double>(Nc);
            fails += pmgemu_transfer(dim, n, p, 1, fine.data(), coarse.data()) != 0;
            fails += pmgemu_transfer(dim, n, p, 0, coarse.data(), fine.data()) != 0;
            if (n <= 3) {
              auto z = std::vector<double>(N);
              fails += pmgemu_coarse_solve(dim, n, p, u.data(), z.data()) != 0;
            }
          }
        }
        std::printf("dim %d p %d hierarchy %d ok\n", dim, p, code);
      }
  // general path (Cartesian vertices through the metric code, mu = 1), paper hierarchies
  for (int dim = 2; dim <= 3; ++dim)
    for (int p = 1; p <= 8; ++p) {
      if (dim == 3 && p > 6) continue;
      std::vector<int> deg;
      for (int x = 1; x < p; x = 2 * x + 1) deg.push_back(x);
      deg.push_back(p);
      std::vector<double> om(deg.size(), 0.6);
      const int n = 2;
      const long N = ipow((long)p * n + 1, dim);
      auto u = rnd(N, 5), b = rnd(N, 6), out = std::vector<double>(N);
      fails += pmgemu_metric_apply(dim, n, p, nullptr, nullptr, 1, u.data(), b.data(), out.data()) != 0;
      for (int it = 1; it <= 2; ++it)
        fails += pmgemu_metric_smooth(dim, n, p, deg.data(), (int)deg.size(), om.data(), it - 1, it, 1, nullptr,
                                      nullptr, u.data(), b.data(), 0, nullptr, nullptr) != 0;
      std::printf("general dim %d p %d ok\n", dim, p);
    }
  std::printf("failures: %d\n", fails);
  return fails != 0;
}
