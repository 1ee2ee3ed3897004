// General-path kernel instantiations for dim = 3, compute float, metric storage bf16.
#include "kernels_metric_impl.h"

namespace pmg {
template struct MetricLaunchers<3, float, bf16>;
}  // namespace pmg
