// Kernels of general hex meshes with stored maps for dim = 3, compute and metric float.
#include "kernels_metric_impl.h"

namespace pmg {
template struct HexLaunchers<3, float>;
}  // namespace pmg
