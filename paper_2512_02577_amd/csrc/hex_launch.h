// Host-side launchers of the kernels of general hex meshes with stored maps
// (kernels_hex_*.hip, setup.hip).
#pragma once

#include "launch.h"

namespace pmg {

// Launchers of general hex meshes with stored maps (metric stored in the compute type);
// instantiated in kernels_hex_*.hip for (3D, 2D) x (double, float).
template <int DIM, typename T>
struct HexLaunchers {
  static size_t patch_bytes(int p);
  static size_t apply_bytes(int p);
  // one color: a.plist holds its a.n_patch patches
  static int smooth(int p, const MetricSmoothArgs<T, T> &a, const Arena &ar, hipStream_t s);
  // one color: a.clist holds its a.n_cells cells
  static int apply(int p, const MetricApplyArgs<T, T> &a, const Arena &ar, hipStream_t s);
  static int apply_init(long n_dofs, bool resid, const unsigned char *bnd, const T *b, const T *u, T *out,
                        hipStream_t s);
};

// invD[patch * (2q-1)^d + e] = omega / (patch diagonal), stored as S, for the np patches of
// a general hex mesh whose cells come from the stored lists pcells (2^d per patch)
template <typename S>
int launch_patch_invdiag_list(int dim, int q, long np, const int32_t *pcells, double omega, const double *cdiag,
                              S *invD, hipStream_t s);

}  // namespace pmg
