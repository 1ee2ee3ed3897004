// Host setup of general hexahedral (2D: quadrilateral) meshes given as cell lists with
// stored DoF maps: consistent cell orientation, the Dirichlet boundary, the vertex
// patches with their stored closure maps, and DSATUR colorings of the patches and of
// the cells (Sec. 3: patches are identified at setup and work on their cells' DoF
// indices; Sec. 4.4: DSATUR coloring of the patches).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pmg {

struct HexHost {
  int dim = 3, p = 1;
  long n_vertices = 0, n_cells = 0, n_dofs = 0;
  std::vector<double> xyz;       // dim per vertex
  std::vector<int32_t> cverts;   // 2^d corners per cell, in the common frame
  std::vector<int32_t> cdofs;    // (p+1)^d nodes per cell, in the common frame
  std::vector<uint8_t> bnd;      // per node: on a face that belongs to one cell
  std::vector<int32_t> pvert;    // per patch: its vertex (ascending)
  std::vector<int32_t> pcells;   // per patch: 2^d cells, block position dx + 2 dy + 4 dz
  std::vector<int32_t> pmap;     // per patch: (2p+1)^d closure nodes, x fastest; -1 on the boundary
  std::vector<int32_t> pcolor, ccolor;
  std::vector<int32_t> plist, clist;  // patches / cells grouped by color, inside a color by smallest node
  std::vector<int32_t> pfirst, cfirst;  // offsets of the colors in plist / clist (n_colors + 1)
  int reflected = 0;             // 1 if the common frame was mirrored to make det J > 0
};

// DSATUR (Brelaz 1979) on an adjacency list: repeatedly colors the uncolored vertex with
// the most distinct neighbour colors, ties to the most uncolored neighbours, then to the
// lowest index, with the smallest color no neighbour has.  Returns the number of colors.
int dsatur(const std::vector<std::vector<int32_t>> &adj, std::vector<int32_t> &color);

// Builds everything above from the caller's arrays (validated).  Returns 0, or a
// negative PMG status with a message in err.
int hex_build(int dim, int p, long n_vertices, const double *xyz, long n_cells, const int32_t *cell_vertices,
              long n_dofs, const int32_t *cell_dofs, HexHost &h, std::string &err);

}  // namespace pmg
