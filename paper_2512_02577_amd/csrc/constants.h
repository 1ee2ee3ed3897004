// Compile-time launch shapes shared by the host setup and the kernels.
#pragma once

namespace pmg {

// Cells per direction of one operator-apply tile: the tile owns p*tc nodes per direction
// and reads p*(tc+1)+1, chosen so that the owned extent is 7..12 nodes.
constexpr int tile_cells(int p) { return p == 1 ? 8 : p == 2 ? 4 : p == 3 ? 3 : p <= 6 ? 2 : 1; }

// xy tile (TX x TY cells), planes per group (G) and lanes of the 3D operator apply that
// marches in z, by degree.  The xy input (tile and one halo cell per side) has 289 to 625 z
// columns, one per lane (two at p <= 4 on 256 lanes); the y and x contractions run on G of a
// layer's P planes at a time.  Degrees <= 4 fit three or four workgroups per CU in FP64; from
// degree 6 on the registers of the z window allow only one or two per CU whatever the LDS,
// so the whole layer is one group (fewer barriers per layer).
constexpr int march_tile(int p) { return p == 1 ? 16 : p == 2 ? 8 : p == 3 ? 5 : p == 4 ? 4 : p == 5 ? 3 : 2; }
constexpr int march_tile_y(int p) { return p == 1 ? 16 : p == 2 ? 8 : p == 3 ? 5 : p == 4 ? 3 : p == 5 ? 3 : 2; }
constexpr int march_group(int p) { return p; }
constexpr int march_threads(int p) { return p <= 4 ? 256 : p == 5 ? 512 : p == 6 ? 384 : p == 7 ? 512 : 640; }
// Workgroups a marching apply aims for (the z segments get shorter until it has them).
constexpr int kMarchBlocks = 4096;

// Tiles per direction and cell layers per segment of the marching apply: segments are added
// until the launch has about `target` workgroups, or every layer is a segment of its own.
inline void march_geometry(int n, int tx, int ty, int target, int &mx, int &my, int &nseg, int &zc) {
  mx = (n + tx - 1) / tx;
  my = (n + ty - 1) / ty;
  const int nxy = mx * my;
  int s = (target + nxy - 1) / nxy;
  s = s < 1 ? 1 : (s > n ? n : s);
  zc = (n + s - 1) / s;
  nseg = (n + zc - 1) / zc;
}

// Threads of the coarse-solve workgroup.
constexpr int kCoarseThreads = 512;

}  // namespace pmg
