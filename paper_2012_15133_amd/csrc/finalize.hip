// Single-workgroup kernel that closes a step (the SAV scalar solve) when it is not
// done inside the next update kernel, and closes the start-up, query and
// end-of-run passes.  A separate launch rather than the last workgroup of the
// forward pass: publishing the partial sums from inside that kernel would need an
// agent-scope release in every workgroup, which on a multi-XCD part writes back
// the L2 each time.
#include "kernels.hpp"
#include "launch.hpp"

namespace spfc {

// One workgroup per member of the batch (blockIdx.x).
__global__ void __launch_bounds__(1024) k_finalize(FinalizeArgs p) {
    const int mem = blockIdx.x;
    const Geo geo = p.geos[mem];
    if (p.mode == FIN_STEP) {
        const FinishIn fi = member_fin(p.fi, mem);
        // the forward pass folded the real-space partials into its own (NPART_PF per
        // workgroup: p1, p2, p_psi, the E_1 slice); E: the energy norms
        double sPE[NPART_PF + NPART_E];
        block_sum_pair<NPART_PF, NPART_E>(fi.partP, fi.nPE, fi.partE, fi.nPE, sPE);
        if (threadIdx.x == 0) {
            const double sP[NPART_P] = {sPE[0], sPE[1], sPE[2]};
            double sE[NPART_E];
            for (int i = 0; i < NPART_E; ++i) sE[i] = sPE[NPART_PF + i];
            finish_step(fi, sPE[3], sE, sP, p.a0, p.a1, p.a2, p.dt, geo);
        }
        return;
    }
    double sQB[NPART_E + 1];
    block_sum_pair<NPART_E, 1>(p.partQ + (size_t)mem * p.nQ * NPART_E, p.nQ, p.partB + (size_t)mem * p.nB, p.nB,
                               sQB);
    if (threadIdx.x != 0) return;
    DevScalars* sc = p.sc + mem;
    Record* hist = p.hist + (size_t)mem * p.hist_cap;
    const double n0 = geo.pscale * sQB[0], n1 = geo.pscale * sQB[1];
    const double mean = sQB[4] * geo.inv_npts;
    unsigned int fl = sc->flags;
    if (p.mode == FIN_STATE) {
        // record of the state reached by the last update: energy of (X, Y, r^n, r^{n-1})
        const double rn = sc->r_n, rnm1 = sc->r_nm1;
        const double energy = pair_energy(n0, n1, rn, rnm1, geo.pscale * sQB[5], p.dt, geo);
        if (!isfinite(energy)) fl |= FLAG_NONFINITE;
        if (p.check_rise && energy > sc->energy_prev * (1.0 + p.energy_tol)) fl |= FLAG_ENERGY_RISE;
        const long long step = sc->step_x;
        Record* rc = hist + (step % p.hist_cap);
        rc->energy = energy;
        rc->mean = mean;
        rc->r = rn;
        sc->energy_prev = energy;
        sc->mean = mean;
        sc->last_record = step;
    } else {
        const double E1 = geo.cell * sQB[NPART_E] + geo.e1_const;
        if (!isfinite(E1)) fl |= FLAG_NONFINITE;
        sc->q_E1 = E1;
        sc->q_norm[0] = n0;
        sc->q_norm[1] = n1;
        sc->q_norm[2] = geo.pscale * sQB[2];
        sc->q_norm[3] = geo.pscale * sQB[3];
        sc->q_norm[4] = geo.pscale * sQB[5];
        sc->mean = mean;
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

hipError_t launch_finalize(const FinalizeArgs& a, int members, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(members), dim3(1024), 0, st, a);
    return hipGetLastError();
}

}  // namespace spfc
