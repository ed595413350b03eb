// Single-workgroup reduction that closes the start-up, query and end-of-run
// passes (the per-step reduction lives in the last workgroup of k_spec_fwd).
#include "kernels.hpp"
#include "launch.hpp"

namespace spfc {

// ------------------------------------------------------------------ finalize (one workgroup)

__global__ void __launch_bounds__(256) k_finalize(FinalizeArgs p) {
    double sA[4], sB[1];
    block_sum_partials<4>(p.partA, p.nA, sA);
    block_sum_partials<1>(p.partB, p.nB, sB);
    if (threadIdx.x != 0) return;
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
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace spfc
