// General-path kernel instantiations for dim = 2, compute double, metric storage double.
#include "kernels_metric_impl.h"

namespace pmg {
template struct MetricLaunchers<2, double, double>;
}  // namespace pmg
