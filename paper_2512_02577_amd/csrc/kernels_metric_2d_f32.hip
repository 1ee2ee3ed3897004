// General-path kernel instantiations for dim = 2, compute float, metric storage float.
#include "kernels_metric_impl.h"

namespace pmg {
template struct MetricLaunchers<2, float, float>;
}  // namespace pmg
