// Kernel instantiations for dim = 2, float.
#include "kernels_impl.h"

namespace pmg {
template struct Launchers<2, float>;
}  // namespace pmg
