// Kernel instantiations for dim = 3, float.
#include "kernels_impl.h"

namespace pmg {
template struct Launchers<3, float>;
}  // namespace pmg
