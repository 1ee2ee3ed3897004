// Host-side geometry of the general path (see geometry.h).
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <thread>

namespace pmg {

namespace {

template <typename F>
void parallel_for(long n, int threads, F f) {
  threads = (int)std::max<long>(1, std::min<long>(threads, n));
  std::vector<std::thread> pool;
  const long chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    const long b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    pool.emplace_back([=]() {
      for (long i = b; i < e; ++i) f(i);
    });
  }
  for (auto &th : pool) th.join();
}

}  // namespace

QTab make_qtab(int q) {
  QTab t;
  t.q = q;
  t.nq = q + 1;
  const int nq = t.nq, k = q + 1;
  dvec z = gauss_lobatto(q), xg, wg;
  gauss_legendre(nq, xg, wg);
  t.B.assign((size_t)nq * k, 0.0);
  t.BT.assign((size_t)k * nq, 0.0);
  t.Dq.assign((size_t)nq * nq, 0.0);
  t.DqT.assign((size_t)nq * nq, 0.0);
  for (int g = 0; g < nq; ++g)
    for (int a = 0; a < k; ++a) {
      t.B[(size_t)g * k + a] = lagrange(z, a, xg[g]);
      t.BT[(size_t)a * nq + g] = t.B[(size_t)g * k + a];
    }
  for (int g = 0; g < nq; ++g)
    for (int h = 0; h < nq; ++h) {
      t.Dq[(size_t)g * nq + h] = lagrange_d(xg, h, xg[g]);
      t.DqT[(size_t)h * nq + g] = t.Dq[(size_t)g * nq + h];
    }
  const int NQ = 2 * nq, E = 2 * q + 1, e = 2 * q - 1;
  t.Bpc.assign((size_t)NQ * E, 0.0);
  for (int r = 0; r < NQ; ++r) {
    const int cell = r / nq, g = r % nq;
    for (int a = 0; a < k; ++a) t.Bpc[(size_t)r * E + cell * q + a] = t.B[(size_t)g * k + a];
  }
  t.Bpi.assign((size_t)NQ * e, 0.0);
  t.BpiT.assign((size_t)e * NQ, 0.0);
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < e; ++c) {
      t.Bpi[(size_t)r * e + c] = t.Bpc[(size_t)r * E + c + 1];
      t.BpiT[(size_t)c * NQ + r] = t.Bpi[(size_t)r * e + c];
    }
  t.Dqp.assign((size_t)NQ * NQ, 0.0);
  t.DqpT.assign((size_t)NQ * NQ, 0.0);
  for (int cell = 0; cell < 2; ++cell)
    for (int g = 0; g < nq; ++g)
      for (int h = 0; h < nq; ++h) {
        const double v = t.Dq[(size_t)g * nq + h];
        t.Dqp[(size_t)(cell * nq + g) * NQ + cell * nq + h] = v;
        t.DqpT[(size_t)(cell * nq + h) * NQ + cell * nq + g] = v;
      }
  return t;
}

dvec cartesian_vertices(int dim, int n) {
  const long nv = dim == 3 ? (long)(n + 1) * (n + 1) * (n + 1) : (long)(n + 1) * (n + 1);
  dvec v((size_t)nv * dim);
  for (long i = 0; i < nv; ++i) {
    long r = i;
    for (int a = 0; a < dim; ++a) {
      v[(size_t)i * dim + a] = (double)(r % (n + 1)) / n;
      r /= (n + 1);
    }
  }
  return v;
}

dvec level_vertices(int dim, int n, const dvec &fine, int nl) {
  const int s = n / nl;
  const long nv = dim == 3 ? (long)(nl + 1) * (nl + 1) * (nl + 1) : (long)(nl + 1) * (nl + 1);
  dvec v((size_t)nv * dim);
  for (long i = 0; i < nv; ++i) {
    long r = i, fi = 0, stride = 1;
    for (int a = 0; a < dim; ++a) {
      fi += (r % (nl + 1)) * s * stride;
      r /= (nl + 1);
      stride *= (n + 1);
    }
    for (int a = 0; a < dim; ++a) v[(size_t)i * dim + a] = fine[(size_t)fi * dim + a];
  }
  return v;
}

namespace {

// corners of cell c (lexicographic offsets, x fastest) -> X[corner][axis]
void cell_corners(int dim, int n, const dvec &verts, long c, double X[8][3]) {
  long r = c;
  int ci[3] = {0, 0, 0};
  for (int a = 0; a < dim; ++a) {
    ci[a] = (int)(r % n);
    r /= n;
  }
  const int nc = 1 << dim;
  for (int k = 0; k < nc; ++k) {
    long idx = 0, stride = 1;
    for (int a = 0; a < dim; ++a) {
      idx += (ci[a] + ((k >> a) & 1)) * stride;
      stride *= (n + 1);
    }
    for (int a = 0; a < dim; ++a) X[k][a] = verts[(size_t)idx * dim + a];
  }
}

// image and Jacobian of the multilinear map at reference point xi
void map_point(int dim, const double X[8][3], const double xi[3], double x[3], double J[3][3]) {
  for (int i = 0; i < 3; ++i) {
    x[i] = 0.0;
    for (int j = 0; j < 3; ++j) J[i][j] = 0.0;
  }
  const int nc = 1 << dim;
  for (int k = 0; k < nc; ++k) {
    double lam = 1.0, dl[3] = {1.0, 1.0, 1.0};
    for (int a = 0; a < dim; ++a) {
      const int o = (k >> a) & 1;
      const double val = o ? xi[a] : 1.0 - xi[a], der = o ? 1.0 : -1.0;
      lam *= val;
      for (int b = 0; b < dim; ++b) dl[b] *= (a == b) ? der : val;
    }
    for (int i = 0; i < dim; ++i) {
      x[i] += lam * X[k][i];
      for (int j = 0; j < dim; ++j) J[i][j] += X[k][i] * dl[j];
    }
  }
}

}  // namespace

void gauss_points(int dim, int n, const dvec &verts, int q, dvec &out) {
  const int nq = q + 1;
  dvec xg, wg;
  gauss_legendre(nq, xg, wg);
  const long ncell = dim == 3 ? (long)n * n * n : (long)n * n;
  const int nqd = dim == 3 ? nq * nq * nq : nq * nq;
  out.assign((size_t)ncell * nqd * dim, 0.0);
  for (long c = 0; c < ncell; ++c) {
    double X[8][3];
    cell_corners(dim, n, verts, c, X);
    for (int g = 0; g < nqd; ++g) {
      const double xi[3] = {xg[g % nq], xg[(g / nq) % nq], dim == 3 ? xg[g / (nq * nq)] : 0.0};
      double x[3], J[3][3];
      map_point(dim, X, xi, x, J);
      for (int a = 0; a < dim; ++a) out[((size_t)c * nqd + g) * dim + a] = x[a];
    }
  }
}

bool metric(int dim, int n, const dvec &verts, int q, const double *a, dvec &G, int threads) {
  const long ncell = dim == 3 ? (long)n * n * n : (long)n * n;
  return metric_cells(
      dim, ncell, [&](long c, double X[8][3]) { cell_corners(dim, n, verts, c, X); }, q, a, G, threads);
}

bool metric_cells(int dim, long ncell, const std::function<void(long, double[8][3])> &corners, int q,
                  const double *a, dvec &G, int threads) {
  const int nq = q + 1, nc = metric_components(dim);
  dvec xg, wg;
  gauss_legendre(nq, xg, wg);
  const int nqd = dim == 3 ? nq * nq * nq : nq * nq;
  G.assign((size_t)ncell * nqd * nc, 0.0);
  std::vector<char> bad(ncell, 0);
  parallel_for(ncell, threads, [&](long c) {
    double X[8][3];
    corners(c, X);
    for (int g = 0; g < nqd; ++g) {
      const int gx = g % nq, gy = (g / nq) % nq, gz = dim == 3 ? g / (nq * nq) : 0;
      const double xi[3] = {xg[gx], xg[gy], dim == 3 ? xg[gz] : 0.0};
      const double w = wg[gx] * wg[gy] * (dim == 3 ? wg[gz] : 1.0);
      double x[3], J[3][3];
      map_point(dim, X, xi, x, J);
      double Ji[3][3], det;
      if (dim == 3) {
        det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
              J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
      } else {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        Ji[0][0] = J[1][1] / det;
        Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det;
        Ji[1][1] = J[0][0] / det;
      }
      if (!(det > 0.0)) bad[c] = 1;
      const double s = w * std::fabs(det) * (a ? a[(size_t)c * nqd + g] : 1.0);
      auto M = [&](int k, int l) {  // (J^{-1} J^{-T})[k][l]
        double v = 0.0;
        for (int m = 0; m < dim; ++m) v += Ji[k][m] * Ji[l][m];
        return s * v;
      };
      double *o = &G[((size_t)c * nqd + g) * nc];
      if (dim == 3) {
        o[0] = M(0, 0); o[1] = M(1, 1); o[2] = M(2, 2);
        o[3] = M(0, 1); o[4] = M(0, 2); o[5] = M(1, 2);
      } else {
        o[0] = M(0, 0); o[1] = M(1, 1); o[2] = M(0, 1);
      }
    }
  });
  for (char b : bad)
    if (b) return false;
  return true;
}

void interior_matrix(int dim, int n, int p, const dvec &G, dvec &A, int threads) {
  const QTab t = make_qtab(p);
  const int nq = t.nq, k = p + 1, nc = metric_components(dim);
  const int nqd = dim == 3 ? nq * nq * nq : nq * nq, nd = dim == 3 ? k * k * k : k * k;
  const long ncell = dim == 3 ? (long)n * n * n : (long)n * n;
  const int mline = p * n + 1, mi = mline - 2;
  const long m = dim == 3 ? (long)mi * mi * mi : (long)mi * mi;
  A.assign((size_t)(m * m), 0.0);
  // reference gradients Tg[(g*nd + i)*dim + kdir] of the nodal basis at the Gauss points
  dvec Tg((size_t)nqd * nd * dim);
  {
    dvec z = gauss_lobatto(p), xg, wg;
    gauss_legendre(nq, xg, wg);
    for (int g = 0; g < nqd; ++g) {
      const int gg[3] = {g % nq, (g / nq) % nq, dim == 3 ? g / (nq * nq) : 0};
      for (int i = 0; i < nd; ++i) {
        const int ii[3] = {i % k, (i / k) % k, dim == 3 ? i / (k * k) : 0};
        for (int kd = 0; kd < dim; ++kd) {
          double v = 1.0;
          for (int a = 0; a < dim; ++a)
            v *= (a == kd) ? lagrange_d(z, ii[a], xg[gg[a]]) : t.B[(size_t)gg[a] * k + ii[a]];
          Tg[((size_t)g * nd + i) * dim + kd] = v;
        }
      }
    }
  }
  // element matrices, then scatter into the interior block (cells in parallel, each
  // thread accumulates into its own slice of rows guarded by cell parity coloring)
  auto node_of = [&](long c, int i) -> long {  // interior index of cell-local node, or -1
    long r = c;
    int ci[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
      ci[a] = (int)(r % n);
      r /= n;
    }
    const int ii[3] = {i % k, (i / k) % k, dim == 3 ? i / (k * k) : 0};
    long idx = 0, stride = 1;
    for (int a = 0; a < dim; ++a) {
      const int gidx = p * ci[a] + ii[a];
      if (gidx == 0 || gidx == mline - 1) return -1;
      idx += (gidx - 1) * stride;
      stride *= mi;
    }
    return idx;
  };
  const int ncolor = 1 << dim;
  for (int col = 0; col < ncolor; ++col) {
    std::vector<long> cells;
    for (long c = 0; c < ncell; ++c) {
      long r = c;
      int cc = 0;
      for (int a = 0; a < dim; ++a) {
        cc |= (int)((r % n) & 1) << a;
        r /= n;
      }
      if (cc == col) cells.push_back(c);
    }
    parallel_for((long)cells.size(), threads, [&](long ci) {
      const long c = cells[ci];
      dvec W((size_t)nqd * nd * dim, 0.0), Ae((size_t)nd * nd, 0.0);
      for (int g = 0; g < nqd; ++g) {
        const double *o = &G[((size_t)c * nqd + g) * nc];
        double M[3][3];
        if (dim == 3) {
          M[0][0] = o[0]; M[1][1] = o[1]; M[2][2] = o[2];
          M[0][1] = M[1][0] = o[3]; M[0][2] = M[2][0] = o[4]; M[1][2] = M[2][1] = o[5];
        } else {
          M[0][0] = o[0]; M[1][1] = o[1]; M[0][1] = M[1][0] = o[2];
        }
        for (int j = 0; j < nd; ++j)
          for (int kd = 0; kd < dim; ++kd) {
            double s = 0.0;
            for (int l = 0; l < dim; ++l) s += M[kd][l] * Tg[((size_t)g * nd + j) * dim + l];
            W[((size_t)g * nd + j) * dim + kd] = s;
          }
      }
      for (int g = 0; g < nqd; ++g)
        for (int i = 0; i < nd; ++i) {
          const double *ti = &Tg[((size_t)g * nd + i) * dim];
          for (int j = 0; j < nd; ++j) {
            const double *wj = &W[((size_t)g * nd + j) * dim];
            double s = 0.0;
            for (int kd = 0; kd < dim; ++kd) s += ti[kd] * wj[kd];
            Ae[(size_t)i * nd + j] += s;
          }
        }
      for (int i = 0; i < nd; ++i) {
        const long gi = node_of(c, i);
        if (gi < 0) continue;
        for (int j = 0; j < nd; ++j) {
          const long gj = node_of(c, j);
          if (gj >= 0) A[(size_t)(gi * m + gj)] += Ae[(size_t)i * nd + j];
        }
      }
    });
  }
}

}  // namespace pmg
