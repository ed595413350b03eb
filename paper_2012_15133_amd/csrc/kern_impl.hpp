// Instantiation of the kernel templates for one precision; included by
// kern_f64.hip and kern_f32.hip, each compiled on its own.
#pragma once

#include "kernels.hpp"
#include "launch.hpp"

namespace spfc {

#define SPFC_SWITCH_N(n, BODY)            \
    switch (n) {                          \
        case 8: { constexpr int NN = 8; BODY; } \
        case 16: { constexpr int NN = 16; BODY; } \
        case 32: { constexpr int NN = 32; BODY; } \
        case 64: { constexpr int NN = 64; BODY; } \
        case 128: { constexpr int NN = 128; BODY; } \
        case 256: { constexpr int NN = 256; BODY; } \
        case 512: { constexpr int NN = 512; BODY; } \
        case 1024: { constexpr int NN = 1024; BODY; } \
        default: return hipErrorInvalidValue; \
    }

template <typename T>
hipError_t Kern<T>::spec_inv(int nl, int dim, const SpecInvArgs<T>& a, const LaunchShape& s, hipStream_t st) {
    SPFC_SWITCH_N(nl, {
        if (dim == 2) hipLaunchKernelGGL((k_spec_inv<T, NN, 2>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
        else hipLaunchKernelGGL((k_spec_inv<T, NN, 3>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
        return hipGetLastError();
    })
}

template <typename T>
hipError_t Kern<T>::real_pass(int nx, int dim, bool fwd, const RealArgs<T>& a, const LaunchShape& s,
                              hipStream_t st) {
    SPFC_SWITCH_N(nx, {
        if (dim == 2) {
            if (fwd) hipLaunchKernelGGL((k_real_pass<T, NN, 2, true>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
            else hipLaunchKernelGGL((k_real_pass<T, NN, 2, false>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
        } else {
            if (fwd) hipLaunchKernelGGL((k_real_pass<T, NN, 3, true>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
            else hipLaunchKernelGGL((k_real_pass<T, NN, 3, false>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
        }
        return hipGetLastError();
    })
}

template <typename T>
hipError_t Kern<T>::spec_fwd(int nl, int dim, int mode, const SpecFwdArgs<T>& a, const LaunchShape& s,
                             hipStream_t st) {
    SPFC_SWITCH_N(nl, {
        if (dim == 2) {
            if (mode == FWD_SOLVE)
                hipLaunchKernelGGL((k_spec_fwd<T, NN, 2, FWD_SOLVE>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
            else
                hipLaunchKernelGGL((k_spec_fwd<T, NN, 2, FWD_GHOST>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
        } else {
            if (mode == FWD_SOLVE)
                hipLaunchKernelGGL((k_spec_fwd<T, NN, 3, FWD_SOLVE>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
            else
                hipLaunchKernelGGL((k_spec_fwd<T, NN, 3, FWD_GHOST>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
        }
        return hipGetLastError();
    })
}

template <typename T>
hipError_t Kern<T>::pass(int nl, int dir, int omode, int c, const PassArgs<T>& a, const LaunchShape& s,
                         hipStream_t st) {
#define SPFC_PASS_CASE(D, OM, CC)                                                                      \
    if (dir == D && omode == OM && c == CC) {                                                        \
        hipLaunchKernelGGL((k_pass<T, NN, D, OM, CC>), dim3(s.grid), dim3(s.block), s.shmem, st, a); \
        return hipGetLastError();                                                                    \
    }
    SPFC_SWITCH_N(nl, {
        SPFC_PASS_CASE(-1, OUT_KEEP, 1)
        SPFC_PASS_CASE(-1, OUT_SWAP, 1)
        SPFC_PASS_CASE(+1, OUT_ROTATE, 1)
        SPFC_PASS_CASE(+1, OUT_SWAP, 1)
        SPFC_PASS_CASE(+1, OUT_SWAP, 3)
        SPFC_PASS_CASE(-1, OUT_SWAP, 3)
        return hipErrorInvalidValue;
    })
#undef SPFC_PASS_CASE
}

template <typename T>
hipError_t Kern<T>::update(int dim, const UpdateArgs<T>& a, int grid, int block, hipStream_t st) {
    if (dim == 2) hipLaunchKernelGGL((k_update<T, 2>), dim3(grid), dim3(block), 0, st, a);
    else hipLaunchKernelGGL((k_update<T, 3>), dim3(grid), dim3(block), 0, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t Kern<T>::r2c_rows(int nx, const RowArgs<T>& a, const LaunchShape& s, hipStream_t st) {
    SPFC_SWITCH_N(nx, {
        hipLaunchKernelGGL((k_r2c_rows<T, NN, double>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
        return hipGetLastError();
    })
}

template <typename T>
hipError_t Kern<T>::c2r_rows(int nx, bool out_fp32, const RowArgs<T>& a, const LaunchShape& s, hipStream_t st) {
    SPFC_SWITCH_N(nx, {
        if (out_fp32) hipLaunchKernelGGL((k_c2r_rows<T, NN, float>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
        else hipLaunchKernelGGL((k_c2r_rows<T, NN, double>), dim3(s.grid), dim3(s.block), s.shmem, st, a);
        return hipGetLastError();
    })
}

#undef SPFC_SWITCH_N

}  // namespace spfc
