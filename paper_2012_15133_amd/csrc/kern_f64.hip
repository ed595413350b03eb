// FP64 instances of the step and transform kernels.
#include "kern_impl.hpp"

namespace spfc {
template struct Kern<double>;
}  // namespace spfc
