// FP32 instances of the step and transform kernels (inner products, energies
// and the SAV scalar stay FP64).
#include "kern_impl.hpp"

namespace spfc {
template struct Kern<float>;
}  // namespace spfc
