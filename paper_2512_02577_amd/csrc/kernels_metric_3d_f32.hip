// General-path kernel instantiations for dim = 3, compute float, metric storage float.
#include "kernels_metric_impl.h"

namespace pmg {
template struct MetricLaunchers<3, float, float>;
}  // namespace pmg
