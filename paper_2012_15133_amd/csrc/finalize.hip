// Single-workgroup reduction that closes every step (the SAV scalar solve) and
// the start-up, query and end-of-run passes.  A separate launch, rather than the
// last workgroup of the forward pass, because publishing the partial sums from
// inside that kernel would need an agent-scope release per workgroup, which on a
// multi-XCD part writes back the L2.
#include "kernels.hpp"
#include "launch.hpp"

namespace spfc {

// ------------------------------------------------------------------ finalize (one workgroup)

// Fixed-order sum of all partials of a step in one sweep: every thread reads its
// fixed subset of the three partial arrays (all loads in flight together), then
// one tree over the workgroup.
__device__ inline void sum_all_partials(const FinalizeArgs& p, double (&sA)[4], double (&sB)[1], double (&sC)[3]) {
    __shared__ double red[8][16];
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int nC = p.mode == FIN_STEP ? p.nC : 0;
    const int n = max(p.nA, max(p.nB, nC));
    constexpr int U = 4;   // indices per thread per sweep, loaded before any is added
    for (int j0 = threadIdx.x; j0 < n; j0 += U * blockDim.x) {
        double v[U][8];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int j = j0 + q * blockDim.x;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[q][i] = j < p.nA ? p.partA[(size_t)4 * j + i] : 0.0;
            v[q][4] = j < p.nB ? p.partB[j] : 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) v[q][5 + i] = j < nC ? p.partC[(size_t)3 * j + i] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] += v[q][i];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = wave_sum(acc[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) red[i][wave] = acc[i];
    }
    __syncthreads();
    double s[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        s[i] = 0.0;
        for (int w = 0; w < nw; ++w) s[i] += red[i][w];
    }
    for (int i = 0; i < 4; ++i) sA[i] = s[i];
    sB[0] = s[4];
    for (int i = 0; i < 3; ++i) sC[i] = s[5 + i];
}

__global__ void __launch_bounds__(1024) k_finalize(FinalizeArgs p) {
    double sA[4], sB[1], sC[3];
    sum_all_partials(p, sA, sB, sC);
    if (threadIdx.x != 0) return;
    if (p.mode == FIN_STEP) {
        finish_step(sB[0], sA, sC, p.sc, p.hist, p.hist_cap, p.step, p.a0, p.a1, p.a2, p.dt, p.check_rise,
                    p.energy_tol, p.geo);
        return;
    }
    const Geo& geo = p.geo;
    DevScalars* sc = p.sc;
    const double E1 = geo.cell * sB[0] + geo.e1_const;
    const double n0 = geo.pscale * sA[0], n1 = geo.pscale * sA[1];
    unsigned int fl = sc->flags;
    if (p.mode == FIN_STATE) {
        // record of the state reached by the last update: energy of (X, Y, r^n, r^{n-1})
        const double rn = sc->r_n, rnm1 = sc->r_nm1;
        const double energy = 0.25 * (n0 + n1) + 0.5 * (rn * rn + (2.0 * rn - rnm1) * (2.0 * rn - rnm1));
        const double mean = sc->mean_raw * geo.inv_npts;
        if (!isfinite(energy)) fl |= FLAG_NONFINITE;
        if (p.check_rise && energy > sc->energy_prev * (1.0 + p.energy_tol)) fl |= FLAG_ENERGY_RISE;
        Record* rc = p.hist + (p.step % p.hist_cap);
        rc->energy = energy;
        rc->mean = mean;
        rc->r = rn;
        sc->energy_prev = energy;
        sc->mean = mean;
        sc->last_record = p.step;
    } else {
        if (!isfinite(E1)) fl |= FLAG_NONFINITE;
        sc->q_E1 = E1;
        sc->q_norm[0] = n0;
        sc->q_norm[1] = n1;
        sc->q_norm[2] = geo.pscale * sA[2];
        sc->q_norm[3] = geo.pscale * sA[3];
        sc->mean = sc->mean_raw * geo.inv_npts;
        const double r = sqrt(E1);
        if (p.mode == FIN_GHOST_R0) {
            sc->r_n = r;
        } else if (p.mode == FIN_GHOST_RM1) {
            sc->r_nm1 = r;
        } else if (p.mode == FIN_RESTART) {
            sc->r_n = r;
            sc->r_nm1 = r;
        }
    }
    sc->flags = fl;
}

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

}  // namespace spfc
