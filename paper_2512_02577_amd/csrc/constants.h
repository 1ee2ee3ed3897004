// Compile-time launch shapes shared by the host setup and the kernels.
#pragma once

namespace pmg {

// Cells per direction of one operator-apply tile: the tile owns p*tc nodes per direction
// and reads p*(tc+1)+1, chosen so that the owned extent is 7..12 nodes.
constexpr int tile_cells(int p) { return p == 1 ? 8 : p == 2 ? 4 : p == 3 ? 3 : p <= 6 ? 2 : 1; }

// Threads of the coarse-solve workgroup.
constexpr int kCoarseThreads = 512;

}  // namespace pmg
