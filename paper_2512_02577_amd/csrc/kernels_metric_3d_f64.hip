// General-path kernel instantiations for dim = 3, compute double, metric storage double.
#include "kernels_metric_impl.h"

namespace pmg {
template struct MetricLaunchers<3, double, double>;
}  // namespace pmg
