// Host-side construction of the 1D operator tables (see host_tables.h).
#include "host_tables.h"

#include "constants.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace pmg {

namespace {

// P_k(x) and P_{k-1}(x) by the three-term recurrence (k >= 1)
void legendre_pair(int k, double x, double &pk, double &pkm1) {
  double p0 = 1.0, p1 = x;
  for (int j = 2; j <= k; ++j) {
    double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  pk = p1;
  pkm1 = p0;
}

// cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row major, destroyed):
// A = V diag(w) V^T, V columns are eigenvectors
void sym_eig(int n, dvec A, dvec &w, dvec &V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a = A[(size_t)i * n + j] * A[(size_t)i * n + j];
        tot += a;
        if (i != j) off += a;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // rows/cols p and q
          double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

dvec sub(const dvec &A, int lda, int r0, int nr, int c0, int nc) {
  dvec out((size_t)nr * nc);
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nc; ++j) out[(size_t)i * nc + j] = A[(size_t)(r0 + i) * lda + (c0 + j)];
  return out;
}

// y = (sum_k K_k (x) M_others) x on an n^dim tensor (x fastest), K and M dense n x n
void kron_apply(int dim, int n, const dvec &K, const dvec &M, const dvec &x, dvec &y) {
  size_t N = 1;
  for (int a = 0; a < dim; ++a) N *= n;
  y.assign(N, 0.0);
  std::vector<int> idx(dim), jdx(dim);
  // direct (small) evaluation: y_I = sum_J prod_a F_a(I_a, J_a); iterate over J per axis
  for (int k = 0; k < dim; ++k) {
    dvec t = x, t2(N);
    for (int a = 0; a < dim; ++a) {
      const dvec &F = (a == k) ? K : M;
      size_t stride = 1;
      for (int b = 0; b < a; ++b) stride *= n;
      for (size_t I = 0; I < N; ++I) {
        int ia = (int)((I / stride) % n);
        size_t base = I - (size_t)ia * stride;
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += F[(size_t)ia * n + j] * t[base + (size_t)j * stride];
        t2[I] = s;
      }
      t.swap(t2);
    }
    for (size_t I = 0; I < N; ++I) y[I] += t[I];
  }
}

}  // namespace

dvec gauss_lobatto(int q) {
  if (q < 1) throw std::invalid_argument("degree must be >= 1");
  dvec x(q + 1);
  for (int j = 0; j <= q; ++j) {
    double t = -std::cos(M_PI * j / q);  // Chebyshev-Lobatto start
    if (j > 0 && j < q) {
      for (int it = 0; it < 100; ++it) {
        double pq, pqm1;
        legendre_pair(q, t, pq, pqm1);
        // f = q (P_{q-1} - t P_q), f' = -q (q+1) P_q
        double dt = (t * pq - pqm1) / ((q + 1.0) * pq);
        t -= dt;
        if (std::fabs(dt) < 1e-16) break;
      }
    }
    x[j] = 0.5 * (t + 1.0);
  }
  x[0] = 0.0;
  x[q] = 1.0;
  std::sort(x.begin(), x.end());
  // exact symmetry about 1/2
  for (int j = 0; j <= q / 2; ++j) {
    double s = 0.5 * (x[j] + (1.0 - x[q - j]));
    x[j] = s;
    x[q - j] = 1.0 - s;
  }
  if (q % 2 == 0) x[q / 2] = 0.5;
  return x;
}

void gauss_legendre(int nq, dvec &x, dvec &w) {
  x.resize(nq);
  w.resize(nq);
  for (int j = 0; j < nq; ++j) {
    double t = -std::cos(M_PI * (j + 0.75) / (nq + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double pn, pnm1;
      legendre_pair(nq, t, pn, pnm1);
      if (nq == 1) { pn = t; pnm1 = 1.0; }
      dp = nq * (t * pn - pnm1) / (t * t - 1.0);
      double dt = pn / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double pn, pnm1;
    legendre_pair(nq, t, pn, pnm1);
    if (nq == 1) { pn = t; pnm1 = 1.0; }
    dp = nq * (t * pn - pnm1) / (t * t - 1.0);
    x[j] = 0.5 * (t + 1.0);
    w[j] = 1.0 / ((1.0 - t * t) * dp * dp);  // 2 / ((1-t^2) P'^2) on [-1,1], halved
  }
}

double lagrange(const dvec &z, int i, double x) {
  double v = 1.0;
  for (int m = 0; m < (int)z.size(); ++m)
    if (m != i) v *= (x - z[m]) / (z[i] - z[m]);
  return v;
}

double lagrange_d(const dvec &z, int i, double x) {
  double s = 0.0;
  for (int k = 0; k < (int)z.size(); ++k) {
    if (k == i) continue;
    double term = 1.0 / (z[i] - z[k]);
    for (int m = 0; m < (int)z.size(); ++m)
      if (m != i && m != k) term *= (x - z[m]) / (z[i] - z[m]);
    s += term;
  }
  return s;
}

void cell_matrices(int q, dvec &K, dvec &M) {
  dvec z = gauss_lobatto(q), xq, wq;
  gauss_legendre(q + 1, xq, wq);
  int k = q + 1;
  K.assign((size_t)k * k, 0.0);
  M.assign((size_t)k * k, 0.0);
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      double sk = 0.0, sm = 0.0;
      for (int g = 0; g < k; ++g) {
        sk += wq[g] * lagrange_d(z, a, xq[g]) * lagrange_d(z, b, xq[g]);
        sm += wq[g] * lagrange(z, a, xq[g]) * lagrange(z, b, xq[g]);
      }
      K[(size_t)a * k + b] = sk;
      M[(size_t)a * k + b] = sm;
    }
}

void line_matrices(int q, int ncell, dvec &K, dvec &M) {
  dvec Kc, Mc;
  cell_matrices(q, Kc, Mc);
  int N = q * ncell + 1;
  K.assign((size_t)N * N, 0.0);
  M.assign((size_t)N * N, 0.0);
  for (int c = 0; c < ncell; ++c)
    for (int a = 0; a <= q; ++a)
      for (int b = 0; b <= q; ++b) {
        K[(size_t)(q * c + a) * N + (q * c + b)] += Kc[(size_t)a * (q + 1) + b];
        M[(size_t)(q * c + a) * N + (q * c + b)] += Mc[(size_t)a * (q + 1) + b];
      }
}

int apply_tile_cells(int p) { return tile_cells(p); }

double patch_lambda_max(int dim, const PLevel &L) {
  // Lanczos with full reorthogonalization on D^{-1/2} A D^{-1/2}
  int n = L.n;
  size_t N = 1;
  for (int a = 0; a < dim; ++a) N *= n;
  if (N == 1) return 1.0;
  int steps = (int)std::min<size_t>(N, 60);
  std::vector<dvec> Q;
  dvec alpha, beta;
  dvec v(N), w, tmp;
  for (size_t i = 0; i < N; ++i) v[i] = 1.0 + 0.37 * std::sin(1.0 + 3.1 * i);
  double nv = 0.0;
  for (double a : v) nv += a * a;
  nv = std::sqrt(nv);
  for (double &a : v) a /= nv;
  for (int k = 0; k < steps; ++k) {
    Q.push_back(v);
    dvec s(N);
    for (size_t i = 0; i < N; ++i) s[i] = v[i] / std::sqrt(L.Dref[i]);
    kron_apply(dim, n, L.Kp, L.Mp, s, tmp);
    w.resize(N);
    for (size_t i = 0; i < N; ++i) w[i] = tmp[i] / std::sqrt(L.Dref[i]);
    double a = 0.0;
    for (size_t i = 0; i < N; ++i) a += w[i] * v[i];
    alpha.push_back(a);
    for (int pass = 0; pass < 2; ++pass)
      for (auto &qv : Q) {
        double d = 0.0;
        for (size_t i = 0; i < N; ++i) d += w[i] * qv[i];
        for (size_t i = 0; i < N; ++i) w[i] -= d * qv[i];
      }
    double b = 0.0;
    for (double x : w) b += x * x;
    b = std::sqrt(b);
    if (b < 1e-12 || k == steps - 1) break;
    beta.push_back(b);
    for (size_t i = 0; i < N; ++i) v[i] = w[i] / b;
  }
  int m = (int)alpha.size();
  dvec T((size_t)m * m, 0.0), ev, V;
  for (int i = 0; i < m; ++i) {
    T[(size_t)i * m + i] = alpha[i];
    if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = beta[i];
  }
  sym_eig(m, T, ev, V);
  return *std::max_element(ev.begin(), ev.end());
}

// apply tile of tc cells per direction: output nodes p*c0 .. p*(c0+tc)-1, input nodes
// p*(c0-1) .. p*(c0+tc)
void apply_tile_tables(int p, int tc, dvec &Kt, dvec &Mt) {
  dvec K, M;
  line_matrices(p, tc + 1, K, M);
  const int NI = p * (tc + 1) + 1, NO = p * tc;
  Kt = sub(K, NI, p, NO, 0, NI);
  Mt = sub(M, NI, p, NO, 0, NI);
}

// Generalized symmetric eigenproblem K s = lambda M s (M positive definite), m x m row
// major: eigenvalues lam and eigenvectors as the columns of S (row major), S^T M S = I.
// Cholesky M = Lc Lc^T, then the symmetric C = Lc^-1 K Lc^-T by cyclic Jacobi, S = Lc^-T Q.
void gen_eig(int m, const dvec &Ki, const dvec &Mi, dvec &lam, dvec &S) {
  dvec Lc((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = Mi[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) s -= Lc[(size_t)i * m + k] * Lc[(size_t)j * m + k];
      Lc[(size_t)i * m + j] = (i == j) ? std::sqrt(s) : s / Lc[(size_t)j * m + j];
    }
  dvec X((size_t)m * m);  // X = Lc^{-1} K
  for (int c = 0; c < m; ++c)
    for (int i = 0; i < m; ++i) {
      double s = Ki[(size_t)i * m + c];
      for (int k = 0; k < i; ++k) s -= Lc[(size_t)i * m + k] * X[(size_t)k * m + c];
      X[(size_t)i * m + c] = s / Lc[(size_t)i * m + i];
    }
  dvec C((size_t)m * m);  // C = X Lc^{-T}: solve Lc C^T = X^T
  for (int r = 0; r < m; ++r)
    for (int i = 0; i < m; ++i) {
      double s = X[(size_t)r * m + i];
      for (int k = 0; k < i; ++k) s -= Lc[(size_t)i * m + k] * C[(size_t)r * m + k];
      C[(size_t)r * m + i] = s / Lc[(size_t)i * m + i];
    }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) {
      double s = 0.5 * (C[(size_t)i * m + j] + C[(size_t)j * m + i]);
      C[(size_t)i * m + j] = C[(size_t)j * m + i] = s;
    }
  dvec Qv;
  sym_eig(m, C, lam, Qv);
  S.assign((size_t)m * m, 0.0);
  for (int c = 0; c < m; ++c)
    for (int i = m - 1; i >= 0; --i) {
      double s = Qv[(size_t)i * m + c];
      for (int k = i + 1; k < m; ++k) s -= Lc[(size_t)k * m + i] * S[(size_t)k * m + c];
      S[(size_t)i * m + c] = s / Lc[(size_t)i * m + i];
    }
}

void build_tables(int dim, int p, const std::vector<int> &degrees, const dvec &omega_override,
                  int n_coarse, Tables &t) {
  t = Tables();
  t.dim = dim;
  t.p = p;
  const int L = (int)degrees.size();
  t.lev.resize(L);
  for (int l = 0; l < L; ++l) {
    PLevel &P = t.lev[l];
    P.q = degrees[l];
    P.n = 2 * P.q - 1;
    dvec K, M;
    line_matrices(P.q, 2, K, M);
    int Nc = 2 * P.q + 1;
    P.Kp = sub(K, Nc, 1, P.n, 1, P.n);
    P.Mp = sub(M, Nc, 1, P.n, 1, P.n);
    size_t N = 1;
    for (int a = 0; a < dim; ++a) N *= P.n;
    P.Dref.resize(N);
    for (size_t I = 0; I < N; ++I) {
      int i = (int)(I % P.n), j = (int)((I / P.n) % P.n), k = (int)(I / ((size_t)P.n * P.n));
      double ki = P.Kp[(size_t)i * P.n + i], mi = P.Mp[(size_t)i * P.n + i];
      double kj = P.Kp[(size_t)j * P.n + j], mj = P.Mp[(size_t)j * P.n + j];
      if (dim == 2) {
        P.Dref[I] = ki * mj + mi * kj;
      } else {
        double kk = P.Kp[(size_t)k * P.n + k], mk = P.Mp[(size_t)k * P.n + k];
        P.Dref[I] = ki * mj * mk + mi * kj * mk + mi * mj * kk;
      }
    }
    if (l > 0) {
      const PLevel &C = t.lev[l - 1];
      dvec zf = gauss_lobatto(P.q), zc = gauss_lobatto(C.q);
      P.Tp.assign((size_t)P.n * C.n, 0.0);
      P.TpT.assign((size_t)C.n * P.n, 0.0);
      for (int o = 0; o < P.n; ++o) {
        int i = o + 1;  // fine closure node
        int s = (i <= P.q) ? 0 : 1;
        double xi = zf[i - s * P.q];
        for (int k = 0; k < C.n; ++k) {
          int kc = k + 1;  // coarse closure node
          double v = 0.0;
          if (kc >= s * C.q && kc <= s * C.q + C.q) v = lagrange(zc, kc - s * C.q, xi);
          P.Tp[(size_t)o * C.n + k] = v;
          P.TpT[(size_t)k * P.n + o] = v;
        }
      }
    }
  }
  t.omega.assign(L, 1.0);
  for (int l = 1; l < L; ++l) {
    if ((int)omega_override.size() > l && omega_override[l] > 0.0)
      t.omega[l] = omega_override[l];
    else
      t.omega[l] = 4.0 / (3.0 * patch_lambda_max(dim, t.lev[l]));
  }
  for (int l = 0; l < L; ++l) {
    PLevel &P = t.lev[l];
    P.invD.resize(P.Dref.size());
    for (size_t I = 0; I < P.Dref.size(); ++I) P.invD[I] = (l == 0 ? 1.0 : t.omega[l]) / P.Dref[I];
  }
  // patch residual matrices (degree p): interior rows, closure columns
  {
    dvec K, M;
    line_matrices(p, 2, K, M);
    int Nc = 2 * p + 1;
    t.Kr = sub(K, Nc, 1, 2 * p - 1, 0, Nc);
    t.Mr = sub(M, Nc, 1, 2 * p - 1, 0, Nc);
  }
  t.tc = apply_tile_cells(p);
  apply_tile_tables(p, t.tc, t.Kt, t.Mt);
  // h-embedding: coarse cell basis at the fine Gauss-Lobatto nodes of its two halves
  {
    dvec z = gauss_lobatto(p);
    t.W1.assign((size_t)(2 * p + 1) * (p + 1), 0.0);
    for (int a = 0; a <= 2 * p; ++a) {
      int s = (a < p) ? 0 : 1;
      double xi = 0.5 * (s + z[a - s * p]);
      for (int b = 0; b <= p; ++b) t.W1[(size_t)a * (p + 1) + b] = lagrange(z, b, xi);
    }
    const int nw = 4 * p - 1;
    t.Wr.assign((size_t)(p + 1) * nw, 0.0);
    for (int a = 1; a <= p - 1; ++a)
      for (int k = 0; k < 2 * p - 1; ++k) t.Wr[(size_t)a * nw + k] = t.W1[(size_t)(k + 1) * (p + 1) + a];
    for (int k = 0; k < nw; ++k) {
      double v;
      if (k < 2 * p - 1) v = t.W1[(size_t)(k + 1) * (p + 1) + p];
      else if (k == 2 * p - 1) v = 1.0;
      else v = t.W1[(size_t)(k - 2 * p + 1) * (p + 1) + 0];
      t.Wr[k] = v;  // class a = 0 (coarse vertex)
    }
  }
  // fast diagonalization of every p-level's patch operator (exact local solve, and the
  // Cartesian-reinforced Richardson preconditioner)
  for (int l = 1; l < L; ++l) {
    PLevel &P = t.lev[l];
    gen_eig(P.n, P.Kp, P.Mp, P.lam, P.S);
    P.ST.assign(P.S.size(), 0.0);
    for (int i = 0; i < P.n; ++i)
      for (int a = 0; a < P.n; ++a) P.ST[(size_t)a * P.n + i] = P.S[(size_t)i * P.n + a];
    size_t N = 1;
    for (int d = 0; d < dim; ++d) N *= P.n;
    P.Linv.resize(N);
    for (size_t I = 0; I < N; ++I) {
      const int i = (int)(I % P.n), j = (int)((I / P.n) % P.n), k = (int)(I / ((size_t)P.n * P.n));
      P.Linv[I] = 1.0 / (P.lam[i] + P.lam[j] + (dim == 3 ? P.lam[k] : 0.0));
    }
  }
  // coarsest mesh: generalized eigenproblem K s = lambda M s of the 1D interior matrices
  {
    dvec K, M;
    line_matrices(p, n_coarse, K, M);
    int Nl = p * n_coarse + 1, m = Nl - 2;
    t.m0 = m;
    gen_eig(m, sub(K, Nl, 1, m, 1, m), sub(M, Nl, 1, m, 1, m), t.lam0, t.S0);
  }
}

}  // namespace pmg
