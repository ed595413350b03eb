// Instantiation of the kernel templates for one precision; included by
// kern_f64.hip and kern_f32.hip, each compiled on its own.
#pragma once

#include "kernels.hpp"
#include <algorithm>

#include "launch.hpp"

#include <type_traits>

namespace spfc {

template <int V>
using IC = std::integral_constant<int, V>;

// Call f(IC<n>, IC<e>) for the line length n and the values per thread e (4, 8 or
// 16; n itself for n = 8).
template <typename F>
hipError_t dispatch_ne(int n, int e, F&& f) {
    switch (n) {
        case 8: return f(IC<8>{}, IC<8>{});
#define SPFC_NE_CASE(NV)                               \
    case NV:                                           \
        if (e == 4) return f(IC<NV>{}, IC<4>{});       \
        if (e == 8) return f(IC<NV>{}, IC<8>{});       \
        return f(IC<NV>{}, IC<16>{});
        SPFC_NE_CASE(16)
        SPFC_NE_CASE(32)
        SPFC_NE_CASE(64)
        SPFC_NE_CASE(128)
        SPFC_NE_CASE(256)
        SPFC_NE_CASE(512)
        SPFC_NE_CASE(1024)
#undef SPFC_NE_CASE
        default: return hipErrorInvalidValue;
    }
}

#define SPFC_NE_CONSTS               \
    constexpr int NN = decltype(nn)::value; \
    constexpr int EE = decltype(ee)::value;

template <typename T>
hipError_t Kern<T>::spec_inv(int nl, int dim, bool stab, bool fin, const SpecInvArgs<T>& a, const LaunchShape& s,
                             hipStream_t st) {
    return dispatch_ne(nl, s.E, [&](auto nn, auto ee) -> hipError_t {
        SPFC_NE_CONSTS
        const dim3 g(s.grid, s.members), b(s.block);
#define SPFC_INV(D, S, F) hipLaunchKernelGGL((k_spec_inv<T, NN, EE, D, S, F>), g, b, s.shmem, st, a)
        if (dim == 2) {
            if (stab && fin) SPFC_INV(2, true, true);
            else if (stab) SPFC_INV(2, true, false);
            else if (fin) SPFC_INV(2, false, true);
            else SPFC_INV(2, false, false);
        } else {
            if (stab && fin) SPFC_INV(3, true, true);
            else if (stab) SPFC_INV(3, true, false);
            else if (fin) SPFC_INV(3, false, true);
            else SPFC_INV(3, false, false);
        }
#undef SPFC_INV
        return hipGetLastError();
    });
}

template <typename T>
hipError_t Kern<T>::real_pass(int nx, int dim, bool fwd, bool beta, const RealArgs<T>& a, const LaunchShape& s,
                              hipStream_t st) {
    return dispatch_ne(nx, s.E, [&](auto nn, auto ee) -> hipError_t {
        SPFC_NE_CONSTS
        const dim3 g(s.grid, s.members), b(s.block);
#define SPFC_REAL(D, F, B) hipLaunchKernelGGL((k_real_pass<T, NN, EE, D, F, B>), g, b, s.shmem, st, a)
        if (dim == 2) {
            if (beta) { if (fwd) SPFC_REAL(2, true, true); else SPFC_REAL(2, false, true); }
            else { if (fwd) SPFC_REAL(2, true, false); else SPFC_REAL(2, false, false); }
        } else {
            if (beta) { if (fwd) SPFC_REAL(3, true, true); else SPFC_REAL(3, false, true); }
            else { if (fwd) SPFC_REAL(3, true, false); else SPFC_REAL(3, false, false); }
        }
#undef SPFC_REAL
        return hipGetLastError();
    });
}

template <typename T>
hipError_t Kern<T>::spec_fwd(int nl, int dim, int mode, bool stab, bool fold, const SpecFwdArgs<T>& a,
                             const LaunchShape& s, hipStream_t st) {
    return dispatch_ne(nl, s.E, [&](auto nn, auto ee) -> hipError_t {
        SPFC_NE_CONSTS
        const dim3 g(s.grid, s.members), b(s.block);
#define SPFC_FWD(D, M, S, F) hipLaunchKernelGGL((k_spec_fwd<T, NN, EE, D, M, S, F>), g, b, s.shmem, st, a)
#define SPFC_FWD_DIM(D)                                                                    \
    if (mode == FWD_GHOST) SPFC_FWD(D, FWD_GHOST, false, false);                           \
    else if (mode == FWD_SOLVE_FORCED) {                                                   \
        if (fold) SPFC_FWD(D, FWD_SOLVE_FORCED, false, true);                              \
        else SPFC_FWD(D, FWD_SOLVE_FORCED, false, false);                                  \
    } else if (stab) {                                                                     \
        if (fold) SPFC_FWD(D, FWD_SOLVE, true, true);                                      \
        else SPFC_FWD(D, FWD_SOLVE, true, false);                                          \
    } else {                                                                               \
        if (fold) SPFC_FWD(D, FWD_SOLVE, false, true);                                     \
        else SPFC_FWD(D, FWD_SOLVE, false, false);                                         \
    }
        if (dim == 2) {
            SPFC_FWD_DIM(2)
        } else {
            SPFC_FWD_DIM(3)
        }
#undef SPFC_FWD_DIM
#undef SPFC_FWD
        return hipGetLastError();
    });
}

template <typename T>
hipError_t Kern<T>::pass(int nl, int dir, int omode, int c, const PassArgs<T>& a, const LaunchShape& s,
                         hipStream_t st) {
#define SPFC_PASS_CASE(D, OM, CC)                                                                      \
    if (dir == D && omode == OM && c == CC) {                                                        \
        hipLaunchKernelGGL((k_pass<T, NN, EE, D, OM, CC>), dim3(s.grid, s.members), dim3(s.block), s.shmem, st, a); \
        return hipGetLastError();                                                                    \
    }
    return dispatch_ne(nl, s.E, [&](auto nn, auto ee) -> hipError_t {
        SPFC_NE_CONSTS
        SPFC_PASS_CASE(-1, OUT_KEEP, 1)
        SPFC_PASS_CASE(-1, OUT_SWAP, 1)
        SPFC_PASS_CASE(+1, OUT_ROTATE, 1)
        SPFC_PASS_CASE(+1, OUT_SWAP, 1)
        return hipErrorInvalidValue;
    });
#undef SPFC_PASS_CASE
}

template <typename T>
hipError_t Kern<T>::ypass(int nl, int dir, const PassArgs<T>& a, const LaunchShape& s, hipStream_t st) {
    return dispatch_ne(nl, s.E, [&](auto nn, auto ee) -> hipError_t {
        SPFC_NE_CONSTS
        const dim3 g(s.grid, s.members), b(s.block);
        if (dir > 0) hipLaunchKernelGGL((k_ypass<T, NN, EE, +1>), g, b, s.shmem, st, a);
        else hipLaunchKernelGGL((k_ypass<T, NN, EE, -1>), g, b, s.shmem, st, a);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t Kern<T>::update(int dim, bool stab, const UpdateArgs<T>& a, int grid, int members, int block,
                           hipStream_t st) {
    const dim3 g(grid, members), b(block);
    if (dim == 2) {
        if (stab) hipLaunchKernelGGL((k_update<T, 2, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_update<T, 2, false>), g, b, 0, st, a);
    } else {
        if (stab) hipLaunchKernelGGL((k_update<T, 3, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_update<T, 3, false>), g, b, 0, st, a);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t Kern<T>::force(const ForceArgs<T>& a, hipStream_t st) {
    const long long blocks = std::min<long long>((a.total + 255) / 256, 4096);
    hipLaunchKernelGGL((k_force<T>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t Kern<T>::r2c_rows(int nx, const RowArgs<T>& a, const LaunchShape& s, hipStream_t st) {
    return dispatch_ne(nx, s.E, [&](auto nn, auto ee) -> hipError_t {
        SPFC_NE_CONSTS
        hipLaunchKernelGGL((k_r2c_rows<T, NN, EE, double>), dim3(s.grid, s.members), dim3(s.block), s.shmem, st, a);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t Kern<T>::c2r_rows(int nx, bool out_fp32, const RowArgs<T>& a, const LaunchShape& s, hipStream_t st) {
    return dispatch_ne(nx, s.E, [&](auto nn, auto ee) -> hipError_t {
        SPFC_NE_CONSTS
        if (out_fp32) hipLaunchKernelGGL((k_c2r_rows<T, NN, EE, float>), dim3(s.grid, s.members), dim3(s.block), s.shmem, st, a);
        else hipLaunchKernelGGL((k_c2r_rows<T, NN, EE, double>), dim3(s.grid, s.members), dim3(s.block), s.shmem, st, a);
        return hipGetLastError();
    });
}

#undef SPFC_NE_CONSTS

}  // namespace spfc
