// Host-side geometry of the general (distorted mesh, variable coefficient) path.
//
// Every cell is the multilinear image of the reference cell [0,1]^d under its 2^d vertices
// (Sec. 4: a Cartesian grid whose interior vertices are moved).  The bilinear form
// a(u, v) = int mu grad u . grad v (eq. bilinear-form with the coefficient of Sec. 3) is
// integrated with the tensor (q+1)-point Gauss rule of each degree q, so the operator
// needs, at every quadrature point, the symmetric metric
//     G = w_q mu(x_q) |det J_q| J_q^{-1} J_q^{-T}
// (the geometry and coefficient folded into one tensor, Sec. 3 stores J^{-1} and det J).
#pragma once

#include <functional>
#include <vector>

#include "host_tables.h"

namespace pmg {

// 1D tables of the metric path for degree q on the reference cell, and their two-cell
// patch versions (patch Gauss points: 2(q+1) per direction, cell 0 first).
struct QTab {
  int q = 0, nq = 0;
  dvec B, BT;         // nq x (q+1) basis values at the Gauss points, and transpose
  dvec Dq, DqT;       // nq x nq collocation derivative on the Gauss points, and transpose
  dvec Bpc;           // 2nq x (2q+1): patch closure nodes -> patch Gauss points
  dvec Bpi, BpiT;     // 2nq x (2q-1): patch interior nodes -> patch Gauss points, transpose
  dvec Dqp, DqpT;     // 2nq x 2nq block-diagonal derivative, transpose
};
QTab make_qtab(int q);

constexpr int metric_components(int dim) { return dim == 3 ? 6 : 3; }

// Vertices of the level with nl cells per direction: the fine vertices at stride n / nl.
dvec level_vertices(int dim, int n, const dvec &fine, int nl);
dvec cartesian_vertices(int dim, int n);

// Physical Gauss points of degree q: n^d cells x (q+1)^d points x d, x fastest.
void gauss_points(int dim, int n, const dvec &verts, int q, dvec &out);

// Metric per Gauss point: n^d cells x (q+1)^d points x (6 | 3) components, ordered
// (xx, yy, zz, xy, xz, yz) in 3D and (xx, yy, xy) in 2D.  a: coefficient per Gauss point
// (same layout, one value) or nullptr for mu = 1.  Returns false on a degenerate cell.
bool metric(int dim, int n, const dvec &verts, int q, const double *a, dvec &G, int threads = 8);
// The same for a list of ncell cells whose corners (lexicographic, x fastest) come from
// corners(c, X); G and a are laid out per listed cell.
bool metric_cells(int dim, long ncell, const std::function<void(long, double[8][3])> &corners, int q,
                  const double *a, dvec &G, int threads = 8);

// Dense interior block of the degree-p operator on a mesh of n cells per direction,
// assembled from element matrices built with the metric G (degree p).  Interior nodes in
// lexicographic order; m = (p n - 1)^d rows, row major.
void interior_matrix(int dim, int n, int p, const dvec &G, dvec &A, int threads = 8);

}  // namespace pmg
