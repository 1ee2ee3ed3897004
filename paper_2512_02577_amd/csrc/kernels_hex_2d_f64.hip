// Kernels of general hex meshes with stored maps for dim = 2, compute and metric double.
#include "kernels_metric_impl.h"

namespace pmg {
template struct HexLaunchers<2, double>;
}  // namespace pmg
