// Bounds- and race-checked run of every emulated kernel body, built with AddressSanitizer
// and UndefinedBehaviorSanitizer (`python -m paper_2512_02577_amd.build --asan`) or with
// ThreadSanitizer (`--tsan`).  Every arena and vector is allocated at its exact size, so an
// out-of-range index in a body aborts the run; each body runs with one lane and with the
// lane counts of the library's launches (one host thread per lane, a barrier for every
// workgroup barrier), so a read or write that is not ordered by a barrier shows up as a
// data race under ThreadSanitizer.  The Cartesian patch bodies also run on the library's
// concatenated table block.
//
//   hostemu_check [quick]      quick: fewer mesh sizes (for the slower sanitizers)
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

extern "C" {
int pmgemu_smooth(int dim, int n, int p, const int *deg, int L, const double *omega, int local, int reinf,
                  int n_iter, int color_dir, double *u, const double *b, int lanes, int one, int tabmode);
int pmgemu_local_solve(int dim, int n, int p, const int *deg, int L, const double *omega, int local, int reinf,
                       int n_iter, int n_blocks, const double *r, double *d, int lanes, int tabmode);
int pmgemu_apply(int dim, int n, int p, int kind, const double *u, const double *b, double *out, int lanes,
                 int zsplit);
int pmgemu_transfer(int dim, int nc, int p, int restrict_, const double *in, double *out);
int pmgemu_coarse_solve(int dim, int n0, int p, const double *r, double *z, int lanes);
int pmgemu_metric_apply(int dim, int n, int p, const double *verts, const double *coef, int resid, const double *u,
                        const double *b, double *out, int lanes);
int pmgemu_metric_smooth(int dim, int n, int p, const int *deg, int L, const double *omega, int full, int n_iter,
                         int color_dir, const double *verts, const double *const *coefs, double *u, const double *b,
                         int nb, const double *r, double *d, int lanes, int one);
}

static std::vector<double> rnd(size_t n, unsigned seed) {
  std::mt19937 g(seed);
  std::uniform_real_distribution<double> d(-1, 1);
  std::vector<double> v(n);
  for (auto &x : v) x = d(g);
  return v;
}

static long ipow(long b, int e) { return e ? b * ipow(b, e - 1) : 1; }

int main(int argc, char **argv) {
  const bool quick = argc > 1 && std::strcmp(argv[1], "quick") == 0;
  int fails = 0;
  auto check = [&](int rc, const char *what, int dim, int p, int n, int lanes) {
    if (rc != 0) {
      std::printf("FAIL %s dim %d p %d n %d lanes %d rc %d\n", what, dim, p, n, lanes, rc);
      ++fails;
    }
  };
  if (argc > 1 && std::strcmp(argv[1], "apply") == 0) {  // the operator applies only, more mesh sizes
    for (int dim = 2; dim <= 3; ++dim)
      for (int p = 1; p <= 8; ++p)
        for (int n : {1, 2, 3, 4, 5, 9, 17}) {
          const long N = ipow((long)p * n + 1, dim);
          if (N > 400000) continue;
          auto u = rnd(N, 1), b = rnd(N, 2), out = std::vector<double>(N);
          for (int lanes = 0; lanes <= 1; ++lanes)
            for (int kind = 0; kind < 3; ++kind)
              for (int zs = 0; zs < 2; ++zs)
                check(pmgemu_apply(dim, n, p, kind, u.data(), b.data(), out.data(), lanes, zs), "apply", dim, p, n,
                      lanes);
          std::printf("apply dim %d p %d n %d done\n", dim, p, n);
          std::fflush(stdout);
        }
    std::printf("failures: %d\n", fails);
    return fails != 0;
  }
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
        const int L = (int)deg.size();
        std::vector<double> om(deg.size(), 0.6);
        for (int n : {2, 3, 5}) {
          if (dim == 3 && p >= 7 && n > 3) continue;
          if (quick && n == 5 && !(dim == 2 || p <= 2)) continue;
          const long N = ipow((long)p * n + 1, dim);
          auto u = rnd(N, 1), b = rnd(N, 2), out = std::vector<double>(N);
          for (int lanes = 0; lanes <= 2; ++lanes) {
            if (quick && lanes == 2 && n > 3) continue;
            // one Richardson step uses the smaller arena: check both sizes; the default local
            // solver also runs in its own compiled variant (one = 1)
            for (int it = 1; it <= 2; ++it)
              for (int full = 0; full < 2; ++full)
                for (int reinf = 0; reinf < 2; ++reinf) {
                  check(pmgemu_smooth(dim, n, p, deg.data(), L, om.data(), full, reinf, it, 1, u.data(), b.data(),
                                      lanes, 0, lanes % 2),
                        "smooth", dim, p, n, lanes);
                  if (it == 1 && full == 0 && reinf == 0)
                    for (int tabmode = 0; tabmode < 2; ++tabmode)
                      check(pmgemu_smooth(dim, n, p, deg.data(), L, om.data(), 0, 0, 1, -1, u.data(), b.data(), lanes,
                                          1, tabmode),
                            "smooth one", dim, p, n, lanes);
                }
            check(pmgemu_smooth(dim, n, p, deg.data(), L, om.data(), 2, 0, 1, 1, u.data(), b.data(), lanes, 0, 1),
                  "smooth direct", dim, p, n, lanes);
          }
          if (dim == 3 && (p == 4 || p == 5))  // the half-lane kernel of large launches (default solver)
            for (int tabmode = 0; tabmode < 2; ++tabmode)
              check(pmgemu_smooth(dim, n, p, deg.data(), L, om.data(), 0, 0, 1, tabmode ? 1 : -1, u.data(), b.data(), 3,
                                  1, tabmode),
                    "smooth half lanes", dim, p, n, 3);
          const long nd = ipow(2 * p - 1, dim), np = ipow(n - 1, dim);
          auto r = rnd(nd * np, 3);
          std::vector<double> d(nd * np);
          for (int lanes = 0; lanes <= 1; ++lanes)
            for (int it = 1; it <= 2; ++it)
              for (int local = 0; local < 3; ++local)
                check(pmgemu_local_solve(dim, n, p, deg.data(), L, om.data(), local, it - 1, it, (int)np, r.data(),
                                         d.data(), lanes, lanes),
                      "local", dim, p, n, lanes);
          if (code == 0) {
            for (int lanes = 0; lanes <= 1; ++lanes) {
              for (int kind = 0; kind < 3; ++kind)
                for (int zs = 0; zs < 2; ++zs)
                  check(pmgemu_apply(dim, n, p, kind, u.data(), b.data(), out.data(), lanes, zs), "apply", dim, p,
                        n, lanes);
            }
            const long Nc = ipow((long)p * n + 1, dim), Nf = ipow(2L * p * n + 1, dim);
            auto fine = rnd(Nf, 4), coarse = std::vector<double>(Nc);
            check(pmgemu_transfer(dim, n, p, 1, fine.data(), coarse.data()), "restrict", dim, p, n, 0);
            check(pmgemu_transfer(dim, n, p, 0, coarse.data(), fine.data()), "prolong", dim, p, n, 0);
            if (n <= 3) {
              auto z = std::vector<double>(N);
              for (int lanes = 0; lanes <= 1; ++lanes)
                check(pmgemu_coarse_solve(dim, n, p, u.data(), z.data(), lanes), "coarse", dim, p, n, lanes);
            }
          }
        }
        std::printf("dim %d p %d hierarchy %d done\n", dim, p, code);
        std::fflush(stdout);
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
      for (int lanes = 0; lanes <= 1; ++lanes) {
        check(pmgemu_metric_apply(dim, n, p, nullptr, nullptr, 1, u.data(), b.data(), out.data(), lanes), "mapply",
              dim, p, n, lanes);
        for (int it = 1; it <= 2; ++it)
          check(pmgemu_metric_smooth(dim, n, p, deg.data(), (int)deg.size(), om.data(), it - 1, it, 1, nullptr,
                                     nullptr, u.data(), b.data(), 0, nullptr, nullptr, lanes, 0),
                "msmooth", dim, p, n, lanes);
        check(pmgemu_metric_smooth(dim, n, p, deg.data(), (int)deg.size(), om.data(), 0, 1, -1, nullptr, nullptr,
                                   u.data(), b.data(), 0, nullptr, nullptr, lanes, 1),
              "msmooth one", dim, p, n, lanes);
      }
      std::printf("general dim %d p %d done\n", dim, p);
      std::fflush(stdout);
    }
  std::printf("failures: %d\n", fails);
  return fails != 0;
}
