// Host setup of general hex meshes with stored maps (see hex_setup.h).
#include "hex_setup.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <queue>
#include <set>
#include <tuple>

#include "host_tables.h"
#include "pmg.h"

namespace pmg {

namespace {

int bad(std::string &err, int code, const char *fmt, long a = 0, long b = 0, long c = 0) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), fmt, a, b, c);
  err = buf;
  return code;
}

struct FaceRec {
  std::array<int32_t, 4> key;  // sorted corner vertices (2D: two, padded with -1)
  int32_t cell;
  int8_t axis, side;           // the face in the cell's input frame
  bool operator<(const FaceRec &o) const {
    return std::tie(key, cell, axis, side) < std::tie(o.key, o.cell, o.axis, o.side);
  }
};

// corner j of the common frame -> corner of the input frame, from a cube symmetry
struct Sym {
  int perm[3] = {0, 1, 2}, flip[3] = {0, 0, 0};
};

Sym sym_of(int dim, const int *lv) {
  Sym s;
  for (int a = 0; a < dim; ++a) {
    const int x = lv[0] ^ lv[1 << a];
    s.perm[a] = x == 1 ? 0 : (x == 2 ? 1 : (x == 4 ? 2 : -1));
    s.flip[a] = s.perm[a] >= 0 ? (lv[0] >> s.perm[a]) & 1 : 0;
  }
  return s;
}

// input-frame index of a node with common-frame coordinates t (k points per axis)
int map_node(int dim, const Sym &s, int k, const int *t) {
  int in[3] = {0, 0, 0};
  for (int a = 0; a < dim; ++a) in[s.perm[a]] = s.flip[a] ? k - 1 - t[a] : t[a];
  return in[0] + k * (in[1] + (dim == 3 ? k * in[2] : 0));
}

double center_det(int dim, const double *X) {  // X[corner * dim + axis], common frame
  double J[3][3] = {{0}};
  const int nc = 1 << dim;
  for (int k = 0; k < nc; ++k)
    for (int a = 0; a < dim; ++a) {
      // d/dxi_a of the multilinear weight at xi = 1/2: +-1/2^(dim-1)
      const double dw = (((k >> a) & 1) ? 1.0 : -1.0) / (double)(1 << (dim - 1));
      for (int i = 0; i < dim; ++i) J[i][a] += X[k * dim + i] * dw;
    }
  if (dim == 2) return J[0][0] * J[1][1] - J[0][1] * J[1][0];
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Items grouped by color; inside a color ordered by key (ties by index).  The order inside
// a color does not change any result (items of one color touch disjoint outputs); ordering
// by the smallest node an item touches lets neighbouring workgroups share cache lines when
// the caller's numbering has locality.
void group_by_color(const std::vector<int32_t> &color, int ncol, const std::vector<int32_t> &key,
                    std::vector<int32_t> &list, std::vector<int32_t> &first) {
  first.assign(ncol + 1, 0);
  for (int32_t c : color) ++first[c + 1];
  for (int i = 0; i < ncol; ++i) first[i + 1] += first[i];
  list.assign(color.size(), 0);
  std::vector<int32_t> pos(first.begin(), first.end() - 1);
  for (size_t i = 0; i < color.size(); ++i) list[pos[color[i]]++] = (int32_t)i;
  for (int c = 0; c < ncol; ++c)
    std::sort(list.begin() + first[c], list.begin() + first[c + 1],
              [&](int32_t a, int32_t b) { return key[a] != key[b] ? key[a] < key[b] : a < b; });
}

}  // namespace

int dsatur(const std::vector<std::vector<int32_t>> &adj, std::vector<int32_t> &color) {
  const long n = (long)adj.size();
  color.assign(n, -1);
  std::vector<std::vector<int32_t>> seen(n);  // distinct neighbour colors, sorted
  std::vector<int32_t> udeg(n);
  // ordered by (saturation desc, uncolored degree desc, index asc)
  std::set<std::tuple<int, int, int32_t>> q;
  for (long v = 0; v < n; ++v) {
    udeg[v] = (int32_t)adj[v].size();
    q.insert({0, -udeg[v], (int32_t)v});
  }
  int ncol = 0;
  while (!q.empty()) {
    const int32_t v = std::get<2>(*q.begin());
    q.erase(q.begin());
    int c = 0;
    for (int32_t s : seen[v]) {  // smallest color not in the sorted list
      if (s == c)
        ++c;
      else if (s > c)
        break;
    }
    color[v] = c;
    ncol = std::max(ncol, c + 1);
    for (int32_t w : adj[v]) {
      if (color[w] >= 0) continue;
      q.erase({-(int)seen[w].size(), -udeg[w], w});
      auto it = std::lower_bound(seen[w].begin(), seen[w].end(), c);
      if (it == seen[w].end() || *it != c) seen[w].insert(it, c);
      --udeg[w];
      q.insert({-(int)seen[w].size(), -udeg[w], w});
    }
  }
  return ncol;
}

int hex_build(int dim, int p, long nv, const double *xyz, long nc, const int32_t *cv_in, long nd,
              const int32_t *cd_in, HexHost &h, std::string &err) {
  if (dim != 2 && dim != 3) return bad(err, PMG_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (p < 1 || p > 8) return bad(err, PMG_ERR_INVALID_ARG, "degree must be in [1, 8]");
  if (nv < 1 || nc < 1 || nd < 1 || nv > INT32_MAX || nc > INT32_MAX || nd > INT32_MAX)
    return bad(err, PMG_ERR_INVALID_ARG, "counts must be in [1, 2^31)");
  const int ncn = 1 << dim, k = p + 1, kd = dim == 3 ? k * k * k : k * k;
  for (long i = 0; i < nv * dim; ++i)
    if (!std::isfinite(xyz[i])) return bad(err, PMG_ERR_INVALID_ARG, "vertex coordinate %ld is not finite", i);
  for (long c = 0; c < nc; ++c) {
    for (int j = 0; j < ncn; ++j) {
      const int32_t v = cv_in[c * ncn + j];
      if (v < 0 || v >= nv) return bad(err, PMG_ERR_INVALID_ARG, "cell %ld lists vertex %ld out of range", c, v);
      for (int i = 0; i < j; ++i)
        if (cv_in[c * ncn + i] == v) return bad(err, PMG_ERR_INVALID_ARG, "cell %ld repeats vertex %ld", c, v);
    }
    for (int j = 0; j < kd; ++j) {
      const int32_t d = cd_in[c * kd + j];
      if (d < 0 || d >= nd) return bad(err, PMG_ERR_INVALID_ARG, "cell %ld lists node %ld out of range", c, d);
    }
  }
  // every node must sit at one place: its Gauss-Lobatto position in each cell listing it
  {
    const dvec z = gauss_lobatto(p);
    std::vector<double> first((size_t)nd * 3, 0.0);
    std::vector<uint8_t> have(nd, 0);
    for (long c = 0; c < nc; ++c) {
      double X[8][3] = {{0}}, diam = 0.0;
      for (int j = 0; j < ncn; ++j)
        for (int a = 0; a < dim; ++a) X[j][a] = xyz[(size_t)cv_in[c * ncn + j] * dim + a];
      for (int a = 0; a < dim; ++a) diam += (X[ncn - 1][a] - X[0][a]) * (X[ncn - 1][a] - X[0][a]);
      const double tol = 1e-9 * std::sqrt(diam);
      for (int e = 0; e < kd; ++e) {
        const int t[3] = {e % k, (e / k) % k, dim == 3 ? e / (k * k) : 0};
        double x[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < ncn; ++j) {
          double w = 1.0;
          for (int a = 0; a < dim; ++a) w *= ((j >> a) & 1) ? z[t[a]] : 1.0 - z[t[a]];
          for (int a = 0; a < dim; ++a) x[a] += w * X[j][a];
        }
        const int32_t d = cd_in[c * kd + e];
        double *f = &first[(size_t)d * 3];
        if (!have[d]) {
          have[d] = 1;
          for (int a = 0; a < dim; ++a) f[a] = x[a];
        } else {
          double dist = 0.0;
          for (int a = 0; a < dim; ++a) dist += (f[a] - x[a]) * (f[a] - x[a]);
          if (std::sqrt(dist) > tol)
            return bad(err, PMG_ERR_INVALID_ARG, "node %ld is listed at two places (cell %ld, local node %ld)", d, c, e);
        }
      }
    }
  }
  h = HexHost{};
  h.dim = dim;
  h.p = p;
  h.n_vertices = nv;
  h.n_cells = nc;
  h.n_dofs = nd;
  h.xyz.assign(xyz, xyz + nv * dim);

  // ---- faces (input frames), sorted by their corner set ----
  const int nf = 2 * dim;
  std::vector<FaceRec> faces;
  faces.reserve((size_t)nc * nf);
  for (long c = 0; c < nc; ++c)
    for (int a = 0; a < dim; ++a)
      for (int s = 0; s < 2; ++s) {
        FaceRec f;
        f.key.fill(-1);
        int m = 0;
        for (int j = 0; j < ncn; ++j)
          if (((j >> a) & 1) == s) f.key[m++] = cv_in[c * ncn + j];
        std::sort(f.key.begin(), f.key.begin() + m);
        f.cell = (int32_t)c;
        f.axis = (int8_t)a;
        f.side = (int8_t)s;
        faces.push_back(f);
      }
  std::sort(faces.begin(), faces.end());
  // neighbour across each (cell, input face): -1 on the boundary
  std::vector<int32_t> nb((size_t)nc * nf, -1);
  std::vector<int8_t> nbface((size_t)nc * nf, -1);
  for (size_t i = 0; i < faces.size();) {
    size_t j = i;
    while (j < faces.size() && faces[j].key == faces[i].key) ++j;
    if (j - i > 2) return bad(err, PMG_ERR_INVALID_ARG, "a face is shared by %ld cells", (long)(j - i));
    if (j - i == 2) {
      const FaceRec &A = faces[i], &B = faces[i + 1];
      if (A.cell == B.cell) return bad(err, PMG_ERR_INVALID_ARG, "cell %ld meets itself", A.cell);
      nb[(size_t)A.cell * nf + 2 * A.axis + A.side] = B.cell;
      nbface[(size_t)A.cell * nf + 2 * A.axis + A.side] = (int8_t)(2 * B.axis + B.side);
      nb[(size_t)B.cell * nf + 2 * B.axis + B.side] = A.cell;
      nbface[(size_t)B.cell * nf + 2 * B.axis + B.side] = (int8_t)(2 * A.axis + A.side);
    }
    i = j;
  }

  // ---- one common frame per face-connected component (breadth first over faces) ----
  std::vector<int> lv((size_t)nc * ncn, -1);  // common corner -> input corner
  std::vector<int32_t> comp(nc, -1);
  int ncomp = 0;
  for (long c0 = 0; c0 < nc; ++c0) {
    if (comp[c0] >= 0) continue;
    for (int j = 0; j < ncn; ++j) lv[c0 * ncn + j] = j;
    comp[c0] = ncomp;
    std::queue<int32_t> qu;
    qu.push((int32_t)c0);
    while (!qu.empty()) {
      const int32_t A = qu.front();
      qu.pop();
      const int *la = &lv[(size_t)A * ncn];
      for (int a = 0; a < dim; ++a)
        for (int s = 0; s < 2; ++s) {
          // the common-frame face (a, s) of A is the input face holding its corners
          int ia = -1, is = -1;
          const int x0 = la[s << a];
          for (int b = 0; b < dim; ++b) {
            bool all = true;
            for (int j = 0; j < ncn; ++j)
              if (((j >> a) & 1) == s && ((la[j] >> b) & 1) != ((x0 >> b) & 1)) all = false;
            if (all) {
              ia = b;
              is = (x0 >> b) & 1;
            }
          }
          if (ia < 0) return bad(err, PMG_ERR_INVALID_ARG, "cell %ld is not a hexahedron", A);
          const int32_t B = nb[(size_t)A * nf + 2 * ia + is];
          if (B < 0) continue;
          const int bface = nbface[(size_t)A * nf + 2 * ia + is], bax = bface / 2;
          int cand[8];
          for (int j = 0; j < ncn; ++j) {
            if (((j >> a) & 1) != s) continue;
            const int32_t v = cv_in[(size_t)A * ncn + la[j]];
            int x = -1;
            for (int t = 0; t < ncn; ++t)
              if (cv_in[(size_t)B * ncn + t] == v) x = t;
            if (x < 0) return bad(err, PMG_ERR_INVALID_ARG, "cells %ld and %ld disagree on a face", A, B);
            cand[j ^ (1 << a)] = x;          // on the shared face, seen from B
            cand[j] = x ^ (1 << bax);        // across B from it
          }
          int *lb = &lv[(size_t)B * ncn];
          if (comp[B] < 0) {
            for (int j = 0; j < ncn; ++j) lb[j] = cand[j];
            comp[B] = ncomp;
            qu.push(B);
          } else {
            for (int j = 0; j < ncn; ++j)
              if (lb[j] != cand[j])
                return bad(err, PMG_ERR_UNSUPPORTED, "cells %ld and %ld cannot share one orientation", A, B);
          }
        }
    }
    ++ncomp;
  }
  // every map must be a symmetry of the cube; mirror components with det J < 0
  std::vector<double> X(ncn * dim);
  std::vector<int> sign(ncomp, 0);
  for (long c = 0; c < nc; ++c) {
    const int *l = &lv[(size_t)c * ncn];
    const Sym sy = sym_of(dim, l);
    for (int j = 0; j < ncn; ++j) {
      int t[3] = {j & 1, (j >> 1) & 1, (j >> 2) & 1};
      if (sy.perm[0] < 0 || sy.perm[1] < 0 || (dim == 3 && sy.perm[2] < 0) || map_node(dim, sy, 2, t) != l[j])
        return bad(err, PMG_ERR_INVALID_ARG, "cell %ld: corners do not form a hexahedron", c);
    }
    for (int j = 0; j < ncn; ++j)
      for (int a = 0; a < dim; ++a) X[j * dim + a] = xyz[(size_t)cv_in[c * ncn + l[j]] * dim + a];
    const double det = center_det(dim, X.data());
    const int sg = det > 0 ? 1 : (det < 0 ? -1 : 0);
    if (sg == 0) return bad(err, PMG_ERR_INVALID_ARG, "cell %ld is degenerate", c);
    if (sign[comp[c]] == 0) sign[comp[c]] = sg;
    if (sign[comp[c]] != sg) return bad(err, PMG_ERR_INVALID_ARG, "cell %ld is inverted against its neighbours", c);
  }
  for (long c = 0; c < nc; ++c)
    if (sign[comp[c]] < 0) {
      int *l = &lv[(size_t)c * ncn];
      for (int j = 0; j < ncn; j += 2) std::swap(l[j], l[j + 1]);  // mirror x of the common frame
      h.reflected = 1;
    }
  h.cverts.resize((size_t)nc * ncn);
  h.cdofs.resize((size_t)nc * kd);
  for (long c = 0; c < nc; ++c) {
    const int *l = &lv[(size_t)c * ncn];
    const Sym sy = sym_of(dim, l);
    for (int j = 0; j < ncn; ++j) h.cverts[(size_t)c * ncn + j] = cv_in[(size_t)c * ncn + l[j]];
    for (int e = 0; e < kd; ++e) {
      const int t[3] = {e % k, (e / k) % k, dim == 3 ? e / (k * k) : 0};
      h.cdofs[(size_t)c * kd + e] = cd_in[(size_t)c * kd + map_node(dim, sy, k, t)];
    }
  }

  // ---- boundary: nodes and vertices on faces of one cell ----
  h.bnd.assign(nd, 0);
  std::vector<uint8_t> vbnd(nv, 0), vused(nv, 0);
  for (long c = 0; c < nc; ++c) {
    for (int j = 0; j < ncn; ++j) vused[cv_in[c * ncn + j]] = 1;
    for (int f = 0; f < nf; ++f) {
      if (nb[(size_t)c * nf + f] >= 0) continue;
      const int a = f / 2, s = f % 2;  // input frame
      for (int j = 0; j < ncn; ++j)
        if (((j >> a) & 1) == s) vbnd[cv_in[c * ncn + j]] = 1;
      for (int e = 0; e < kd; ++e) {
        const int t[3] = {e % k, (e / k) % k, dim == 3 ? e / (k * k) : 0};
        if (t[a] == s * p) h.bnd[cd_in[c * kd + e]] = 1;
      }
    }
  }

  // ---- vertex patches ----
  std::vector<int32_t> vstart(nv + 1, 0), vcells;
  for (long c = 0; c < nc; ++c)
    for (int j = 0; j < ncn; ++j) ++vstart[h.cverts[c * ncn + j] + 1];
  for (long v = 0; v < nv; ++v) vstart[v + 1] += vstart[v];
  vcells.resize(vstart[nv]);
  {
    std::vector<int32_t> pos(vstart.begin(), vstart.end() - 1);
    for (long c = 0; c < nc; ++c)
      for (int j = 0; j < ncn; ++j) vcells[pos[h.cverts[c * ncn + j]]++] = (int32_t)c;
  }
  for (long v = 0; v < nv; ++v)
    if (vused[v] && !vbnd[v]) h.pvert.push_back((int32_t)v);
  const long np = (long)h.pvert.size();
  const int N = 2 * p + 1, Nd = dim == 3 ? N * N * N : N * N;
  h.pcells.assign((size_t)np * ncn, -1);
  h.pmap.assign((size_t)np * Nd, -1);
  for (long q = 0; q < np; ++q) {
    const int32_t v = h.pvert[q];
    const int cnt = vstart[v + 1] - vstart[v];
    if (cnt != ncn)
      return bad(err, PMG_ERR_UNSUPPORTED, "interior vertex %ld has %ld cells; vertex patches need %ld", v, cnt, ncn);
    int32_t *pm = &h.pmap[(size_t)q * Nd];
    for (int i = vstart[v]; i < vstart[v + 1]; ++i) {
      const int32_t c = vcells[i];
      int jc = -1;
      for (int j = 0; j < ncn; ++j)
        if (h.cverts[(size_t)c * ncn + j] == v) jc = j;
      const int bi = (~jc) & (ncn - 1);
      if (h.pcells[(size_t)q * ncn + bi] >= 0)
        return bad(err, PMG_ERR_UNSUPPORTED, "the cells around vertex %ld do not form a 2^d block", v);
      h.pcells[(size_t)q * ncn + bi] = c;
      const int b[3] = {bi & 1, (bi >> 1) & 1, (bi >> 2) & 1};
      for (int e = 0; e < kd; ++e) {
        const int t[3] = {e % k, (e / k) % k, dim == 3 ? e / (k * k) : 0};
        const int X0 = b[0] * p + t[0], Y0 = b[1] * p + t[1], Z0 = dim == 3 ? b[2] * p + t[2] : 0;
        const long idx = X0 + (long)N * (Y0 + (long)N * Z0);
        const int32_t d = h.cdofs[(size_t)c * kd + e];
        if (pm[idx] >= 0 && pm[idx] != d)
          return bad(err, PMG_ERR_INVALID_ARG, "the node map is not conforming around vertex %ld", v);
        pm[idx] = d;
      }
    }
    for (int e = 0; e < Nd; ++e) {
      if (pm[e] < 0) return bad(err, PMG_ERR_INVALID_ARG, "patch of vertex %ld has an unmapped node", v);
      const int i = e % N, j = (e / N) % N, l = dim == 3 ? e / (N * N) : 1;
      const bool inner = i > 0 && i < N - 1 && j > 0 && j < N - 1 && l > 0 && (dim == 2 || l < N - 1);
      if (inner && h.bnd[pm[e]])
        return bad(err, PMG_ERR_INVALID_ARG, "patch of vertex %ld has a boundary node inside", v);
      if (h.bnd[pm[e]]) pm[e] = -1;
    }
  }

  // ---- colorings: patches sharing a cell, cells sharing a vertex ----
  std::vector<std::vector<int32_t>> cpat(nc);
  for (long q = 0; q < np; ++q)
    for (int j = 0; j < ncn; ++j) cpat[h.pcells[(size_t)q * ncn + j]].push_back((int32_t)q);
  std::vector<std::vector<int32_t>> adj(np);
  for (long c = 0; c < nc; ++c)
    for (int32_t a : cpat[c])
      for (int32_t b : cpat[c])
        if (a != b) adj[a].push_back(b);
  for (auto &l : adj) {
    std::sort(l.begin(), l.end());
    l.erase(std::unique(l.begin(), l.end()), l.end());
  }
  const int npc = dsatur(adj, h.pcolor);
  std::vector<int32_t> key(np, INT32_MAX);
  for (long q = 0; q < np; ++q)
    for (int e = 0; e < Nd; ++e) {
      const int32_t d = h.pmap[(size_t)q * Nd + e];
      if (d >= 0 && d < key[q]) key[q] = d;
    }
  group_by_color(h.pcolor, npc, key, h.plist, h.pfirst);
  std::vector<std::vector<int32_t>> cadj(nc);
  for (long c = 0; c < nc; ++c) {
    for (int j = 0; j < ncn; ++j) {
      const int32_t v = h.cverts[c * ncn + j];
      for (int i = vstart[v]; i < vstart[v + 1]; ++i)
        if (vcells[i] != c) cadj[c].push_back(vcells[i]);
    }
    std::sort(cadj[c].begin(), cadj[c].end());
    cadj[c].erase(std::unique(cadj[c].begin(), cadj[c].end()), cadj[c].end());
  }
  const int ncc = dsatur(cadj, h.ccolor);
  key.assign(nc, INT32_MAX);
  for (long c = 0; c < nc; ++c)
    for (int e = 0; e < kd; ++e) key[c] = std::min(key[c], h.cdofs[(size_t)c * kd + e]);
  group_by_color(h.ccolor, ncc, key, h.clist, h.cfirst);
  return 0;
}

}  // namespace pmg
