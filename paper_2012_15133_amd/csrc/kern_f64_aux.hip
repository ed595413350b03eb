// double instances: generic line passes, row transforms, the elementwise update and the forcing.
#include "kern_impl.hpp"

namespace spfc {
template hipError_t Kern<double>::pass(int, int, int, int, const PassArgs<double>&, const LaunchShape&, hipStream_t);
template hipError_t Kern<double>::ypass(int, int, const PassArgs<double>&, const LaunchShape&, hipStream_t);
template hipError_t Kern<double>::update(int, bool, const UpdateArgs<double>&, int, int, int, hipStream_t);
template hipError_t Kern<double>::r2c_rows(int, const RowArgs<double>&, const LaunchShape&, hipStream_t);
template hipError_t Kern<double>::c2r_rows(int, bool, const RowArgs<double>&, const LaunchShape&, hipStream_t);
template hipError_t Kern<double>::force(const ForceArgs<double>&, hipStream_t);
}  // namespace spfc
