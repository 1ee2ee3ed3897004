// Kernel instantiations for dim = 2, double.
#include "kernels_impl.h"

namespace pmg {
template struct Launchers<2, double>;
}  // namespace pmg
