// float instances: generic line passes, row transforms, the elementwise update and the forcing.
#include "kern_impl.hpp"

namespace spfc {
template hipError_t Kern<float>::pass(int, int, int, int, const PassArgs<float>&, const LaunchShape&, hipStream_t);
template hipError_t Kern<float>::ypass(int, int, const PassArgs<float>&, const LaunchShape&, hipStream_t);
template hipError_t Kern<float>::update(int, bool, const UpdateArgs<float>&, int, int, int, hipStream_t);
template hipError_t Kern<float>::r2c_rows(int, const RowArgs<float>&, const LaunchShape&, hipStream_t);
template hipError_t Kern<float>::c2r_rows(int, bool, const RowArgs<float>&, const LaunchShape&, hipStream_t);
template hipError_t Kern<float>::force(const ForceArgs<float>&, hipStream_t);
}  // namespace spfc
