// double instances: spectral forward pass (N, the two Fourier solves, inner products, SAV scalar).
#include "kern_impl.hpp"

namespace spfc {
template hipError_t Kern<double>::spec_fwd(int, int, int, bool, bool, const SpecFwdArgs<double>&, const LaunchShape&,
                                          hipStream_t);
}  // namespace spfc
