// Host-side construction of the 1D operator tables used by the kernels.
//
// On a Cartesian cell of size h the Q_q Laplacian with the (q+1)-point Gauss rule is
// h^{d-2} * sum_k (K along axis k) x (M along the other axes), K and M the 1D reference
// stiffness and mass matrices of the Gauss-Lobatto Lagrange basis (Sec. 3: cellwise
// sum factorization).  Every table below is built from K, M, the Lagrange basis and the
// embedding between degrees or meshes, in float64.
#pragma once

#include <cstdint>
#include <vector>

namespace pmg {

using dvec = std::vector<double>;

// Gauss-Lobatto points of degree q on [0, 1] (q+1 points): the end points and the roots
// of P_q', found by Newton's method on (1 - x^2) P_q'(x) = q (P_{q-1} - x P_q).
dvec gauss_lobatto(int q);
// nq-point Gauss-Legendre rule on [0, 1].
void gauss_legendre(int nq, dvec &x, dvec &w);
double lagrange(const dvec &z, int i, double x);
double lagrange_d(const dvec &z, int i, double x);

// 1D reference cell matrices (unit cell), (q+1) x (q+1), row major.
void cell_matrices(int q, dvec &K, dvec &M);
// Assembled 1D matrices on `ncell` unit cells: (q*ncell+1)^2, row major.
void line_matrices(int q, int ncell, dvec &K, dvec &M);

// Everything one p-level of the local solver needs (reference scale h = 1).
struct PLevel {
  int q = 0;          // degree
  int n = 0;          // interior nodes per direction of a patch: 2q - 1
  dvec Kp, Mp;        // n x n interior patch matrices
  dvec Dref;          // n^dim diagonal of the interior patch operator
  dvec invD;          // n^dim: omega / Dref (level > 0) or 1 / Dref (level 0)
  dvec Tp;            // n x n_coarse embedding from the next coarser p-level (level > 0)
  dvec TpT;           // its transpose, n_coarse x n
  // fast diagonalization of the interior patch operator (level > 0): K S = M S diag(lam),
  // S^T M S = I; S and ST = S^T row major (n x n); Linv = 1 / (lam_i + lam_j (+ lam_k)),
  // n^dim, so that the patch operator's inverse is (S x S x S) diag(Linv) (S x S x S)^T / c
  dvec S, ST, lam, Linv;
};

struct Tables {
  int dim = 3, p = 1;
  std::vector<PLevel> lev;  // coarsest (degree 1) first
  dvec omega;               // per p-level
  dvec Kr, Mr;              // (2p-1) x (2p+1): patch interior rows, closure columns
  int tc = 1;               // cells per direction of one apply tile
  dvec Kt, Mt;              // (p*tc) x (p*(tc+1)+1): apply tile rows, tile-plus-halo columns
  dvec W1;                  // (2p+1) x (p+1): coarse cell basis at the fine nodes inside it
  dvec Wr;                  // (p+1) x (4p-1): restriction weights of a coarse node by class
  // coarsest mesh, exact inverse by fast diagonalization of the interior operator
  int m0 = 0;               // interior nodes per direction on the coarsest mesh
  dvec S0, lam0;            // m0 x m0 eigenvectors (S^T M S = I), eigenvalues of (K, M)
};

int apply_tile_cells(int p);
// 1D tables of an apply tile of tc cells per direction (rows: the tile's owned nodes,
// columns: the tile plus one halo cell below).
void apply_tile_tables(int p, int tc, dvec &Kt, dvec &Mt);

// omega_override: empty for the default 4 / (3 lambda_max(D^{-1} A)) per level.
void build_tables(int dim, int p, const std::vector<int> &degrees, const dvec &omega_override,
                  int n_coarse, Tables &t);

// K s = lambda M s for symmetric K and positive definite M (m x m, row major): eigenvalues
// and the eigenvectors as columns of S, normalized to S^T M S = I.
void gen_eig(int m, const dvec &K, const dvec &M, dvec &lam, dvec &S);

// lambda_max of D^{-1} A on the reference interior patch operator at one level.
double patch_lambda_max(int dim, const PLevel &L);

}  // namespace pmg
