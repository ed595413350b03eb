// float instances: spectral inverse pass (update + gradient + inverse transform).
#include "kern_impl.hpp"

namespace spfc {
template hipError_t Kern<float>::spec_inv(int, int, bool, bool, const SpecInvArgs<float>&, const LaunchShape&,
                                          hipStream_t);
}  // namespace spfc
