// Kernel instantiations for dim = 3, double.
#include "kernels_impl.h"

namespace pmg {
template struct Launchers<3, double>;
}  // namespace pmg
