// float instances: real-space pass (C2R, pointwise SPFC flux, R2C).
#include "kern_impl.hpp"

namespace spfc {
template hipError_t Kern<float>::real_pass(int, int, bool, bool, const RealArgs<float>&, const LaunchShape&, hipStream_t);
}  // namespace spfc
