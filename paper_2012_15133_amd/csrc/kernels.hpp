// HIP kernels of one SAV-BDF2 step of the square phase field crystal equation
// (arXiv 2012.15133, Section 2.3) and of the set-up / query transforms.
//
// Spectral state: the half spectrum (x wavenumbers 0..nx/2) stored [kx][ky]
// (2-D) or [kx][ky][kz] (3-D), last axis contiguous.  One step is
//   2-D: spec_inv (along y) -> real_pass (along x) -> spec_fwd (along y)
//   3-D: spec_inv (z) -> ypass (y) -> real_pass (x) -> ypass (y) -> spec_fwd (z)
// Each symbol is applied by the pass along whose lines it is constant.
// Every kernel reads whole lines along the contiguous axis of its input and
// writes its output with the axes rotated so that the next kernel again reads
// contiguous lines.  Nothing but the state, N and the transform
// intermediates touches HBM; symbols come from indices, in registers.
#pragma once

#include "common.hpp"

namespace spfc {

// ------------------------------------------------------------------ symbols (Section 2.1)

// odd-order symbol 2 pi mt / L, Nyquist mode dropped
__device__ inline double sym1(int m, int n, double k0) {
    if (2 * m == n) return 0.0;
    return k0 * (double)(2 * m < n ? m : m - n);
}
// even-order symbol (2 pi mt / L)^2, Nyquist kept
__device__ inline double sym2(int m, int n, double k0) {
    const double v = k0 * (double)(2 * m <= n ? m : m - n);
    return v * v;
}
// Hermitian weight of x wavenumber kx in a sum over the full spectrum
__device__ inline double hweight(int kx, int nx) { return (kx == 0 || 2 * kx == nx) ? 1.0 : 2.0; }

// ------------------------------------------------------------------ reductions (FP64, fixed order)

// Compiler barrier: no memory access is moved across it (issue order of loads).
__device__ inline void issue_barrier() { asm volatile("" ::: "memory"); }

// Cross-lane moves of a double (two 32-bit halves): a DPP move within rows of 16 lanes
// (CTRL: quad permutation or row mirror) and a read of one lane.
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ inline double lane_value(double v, int lane) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the wave, the same bits in every lane.  Full waves (workgroups of a multiple
// of 64 threads): DPP within each row of 16 lanes (lanes i ^ 1, i ^ 2, then the mirror
// images within 8 and within 16, each step adding a commutative pair), then the four row
// sums in a fixed order.  Otherwise (lanes past the end of the workgroup hold no data) the
// xor butterfly through ds_bpermute.
__device__ inline double wave_sum(double v) {
    if ((blockDim.x & 63) == 0) {
        v += dpp_move<0xB1>(v);    // quad permutation (1, 0, 3, 2)
        v += dpp_move<0x4E>(v);    // quad permutation (2, 3, 0, 1)
        v += dpp_move<0x141>(v);   // row half mirror
        v += dpp_move<0x140>(v);   // row mirror
        return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum NV values over the workgroup and store them at dst[0..NV-1] (thread 0).
template <int NV>
__device__ inline void block_sum_store(double (&acc)[NV], double* dst) {
    __shared__ double red[NV][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = wave_sum(acc[i]);
    __syncthreads();   // an earlier use of `red` is finished
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[i][wave] = acc[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += red[i][w];
            dst[i] = s;
        }
    }
}

// Fixed-order tree over the workgroup of NV per-thread values; the result is
// returned to every thread.
template <int NV>
__device__ inline void block_tree(double (&acc)[NV], double (&out)[NV]) {
    __shared__ double red[NV][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = wave_sum(acc[i]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[i][wave] = acc[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[i][w];
        out[i] = s;
    }
}

// Sum two arrays of per-workgroup partials, a[j*NA + i] (j < na) and
// b[j*NB + i] (j < nb), over the workgroup.  Each thread reads a fixed subset,
// U indices per sweep with every load of a sweep issued before any is added; the
// order of the sums depends only on the workgroup size, so every workgroup of a
// launch gets the same bits.  Result (NA sums of a, then NB sums of b) in every thread.
//
// PairSweep holds one sweep's loads, so that a kernel can issue the first sweep
// before its own loads and reduce while those are in flight (block_sum_pair_from).
template <int NA, int NB>
struct PairSweep {
    static constexpr int U = 4;
    double v[U][NA + NB];
    int j0, na, nb;
    // Every lane loads (entry 0 in place of an index past the end, zeroed when added),
    // so no branch separates these loads from the ones a kernel issues after them and
    // the wait for them does not include those.  Needs a[0..NA) and b[0..NB) readable.
    __device__ inline void load(const double* a, int na_, const double* b, int nb_, int j0_) {
        j0 = j0_;
        na = na_;
        nb = nb_;
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int jj = j0 + q * (int)blockDim.x;
            const size_t ja = jj < na ? jj : 0, jb = jj < nb ? jj : 0;
#pragma unroll
            for (int i = 0; i < NA; ++i) v[q][i] = a[ja * NA + i];
#pragma unroll
            for (int i = 0; i < NB; ++i) v[q][NA + i] = b[jb * NB + i];
        }
    }
    // Pin the loaded values at this point of the program: their wait is placed here,
    // and no use of them (the sums) is moved above it.
    __device__ inline void settle() {
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
            for (int i = 0; i < NA + NB; ++i) asm volatile("" : "+v"(v[q][i]));
    }
    __device__ inline void add_to(double (&acc)[NA + NB]) const {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int jj = j0 + q * (int)blockDim.x;
#pragma unroll
            for (int i = 0; i < NA; ++i) acc[i] += jj < na ? v[q][i] : 0.0;
#pragma unroll
            for (int i = 0; i < NB; ++i) acc[NA + i] += jj < nb ? v[q][NA + i] : 0.0;
        }
    }
};

// block_sum_pair with its first sweep (j0 = threadIdx.x) already loaded into `first`.
// A thread with no index below max(na, nb) adds the zeros of its first sweep, which
// leaves its sums at +0 as the plain loop does.
template <int NA, int NB>
__device__ inline void block_sum_pair_from(const PairSweep<NA, NB>& first, const double* a, int na, const double* b,
                                           int nb, double (&out)[NA + NB]) {
    constexpr int U = PairSweep<NA, NB>::U;
    double acc[NA + NB];
#pragma unroll
    for (int i = 0; i < NA + NB; ++i) acc[i] = 0.0;
    first.add_to(acc);
    const int n = na > nb ? na : nb;
    for (int j0 = threadIdx.x + U * blockDim.x; j0 < n; j0 += U * blockDim.x) {
        PairSweep<NA, NB> s;
        s.load(a, na, b, nb, j0);
        s.add_to(acc);
    }
    block_tree<NA + NB>(acc, out);
}

template <int NA, int NB>
__device__ inline void block_sum_pair(const double* a, int na, const double* b, int nb,
                                      double (&out)[NA + NB]) {
    PairSweep<NA, NB> first;
    first.load(a, na, b, nb, threadIdx.x);
    block_sum_pair_from<NA, NB>(first, a, na, b, nb, out);
}

template <int NV>
__device__ inline void block_sum_partials(const double* part, int n, double (&out)[NV]) {
    double o[NV + 1];
    block_sum_pair<NV, 1>(part, n, part, 0, o);
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = o[i];
}

// ------------------------------------------------------------------ index helpers

// wavenumber indices of element e of spectral line `line` ([a][b][L] layout)
template <int DIM>
__device__ inline void spec_index(int line, int B, int e, int& kx, int& ky, int& kz) {
    if constexpr (DIM == 2) {
        kx = line;
        ky = e;
        kz = 0;
    } else {
        kx = line / B;
        ky = line - kx * B;
        kz = e;
    }
}

template <int DIM>
__device__ inline void spec_symbols(const Geo& g, int kx, int ky, int kz, double& k2, double (&k1)[3]) {
    k1[0] = sym1(kx, g.nx, g.k0x);
    k1[1] = sym1(ky, g.ny, g.k0y);
    k2 = sym2(kx, g.nx, g.k0x) + sym2(ky, g.ny, g.k0y);
    if constexpr (DIM == 3) {
        k1[2] = sym1(kz, g.nz, g.k0z);
        k2 += sym2(kz, g.nz, g.k0z);
    } else {
        k1[2] = 0.0;
    }
}

// Energy partials of the pair (X, Y) at one mode: ||L^1/2 X||^2, ||L^1/2 (2X - Y)||^2,
// ||X||^2, ||Delta X||^2 with the Hermitian weight (modified energy, eq. discrete
// energy; E_N, eq. energy-discrete-spectral), Re X(0) for the mean, and
// <X - Y, -Delta_N (X - Y)> for the extra term of the stabilized scheme's energy.
template <typename T, bool STAB>
__device__ inline void pair_partials(cpx<T> X, cpx<T> Y, int kx, double k2, bool zero_mode, const Geo& geo,
                                     double (&acc)[NPART_E]) {
    const double w = hweight(kx, geo.nx);
    const double Lk = geo.a + k2 * k2;
    const double xx = (double)X.x * X.x + (double)X.y * X.y;
    const double zx = 2.0 * X.x - Y.x, zy = 2.0 * X.y - Y.y;
    acc[0] += w * Lk * xx;
    acc[1] += w * Lk * (zx * zx + zy * zy);
    acc[2] += w * xx;
    acc[3] += w * k2 * k2 * xx;
    if (zero_mode) acc[4] += (double)X.x;
    if constexpr (STAB) {
        const double dx = (double)X.x - Y.x, dy = (double)X.y - Y.y;
        acc[5] += w * k2 * (dx * dx + dy * dy);
    }
}

// Store the energy partials of a workgroup: all NPART_E sums for the stabilized
// kernels, else the first five and a zero (the same layout, without the work).
template <bool STAB>
__device__ inline void store_energy_partials(double (&acc)[NPART_E], double* dst) {
    if constexpr (STAB) {
        block_sum_store<NPART_E>(acc, dst);
    } else {
        double a5[NPART_E - 1];
#pragma unroll
        for (int i = 0; i < NPART_E - 1; ++i) a5[i] = acc[i];
        block_sum_store<NPART_E - 1>(a5, dst);
        if (threadIdx.x == 0) dst[NPART_E - 1] = 0.0;
    }
}

// Symbol of the step operator, A(k) = a0 + dt |k|^2 (a + |k|^4) (eq. solver-1), plus
// stab dt^2 |k|^4 for the stabilized scheme, whose regularization -A dt Delta_N
// (phi^{n+1} - phi^n) in mu also adds stab dt^2 |k|^4 phi^n to the right-hand side.
template <bool STAB>
__device__ inline double stab_sym(const Geo& g, double dt, double k2) {
    if constexpr (STAB) return g.stab * dt * dt * k2 * k2;
    return 0.0;
}

// Stabilized modified energy: the energy of Theorem 3.1 plus (A dt / 4) <X - Y, -Delta_N (X - Y)>.
__device__ inline double pair_energy(double n0, double n1, double rn, double rnm1, double dgrad, double dt,
                                     const Geo& g) {
    return 0.25 * (n0 + n1) + 0.5 * (rn * rn + (2.0 * rn - rnm1) * (2.0 * rn - rnm1)) +
           0.25 * g.stab * dt * dgrad;
}

// xi = r^{n+1} / sqrt(E_1) from the reduced sums (kept out of line so that every
// caller evaluates it with the same instructions and gets the same bits).
// Section 2.3 in this form: with phi^{n+1} = dt xi b1 + b2, b1 = A^-1 Delta N,
// b2 = A^-1 psi, the r equation (eq. scheme-SAV-1, second line) gives
//   xi = [rho + (a0 p2 - p_psi) / (2S)] / [a0 (S - dt p1 / (2S))],
// p1 = <N, b1> <= 0 (eq. solver-5), p2 = <N, b2>, p_psi = <N, psi>, S = sqrt(E_1),
// rho = a1 r^n + a2 r^{n-1}.
__device__ __noinline__ double sav_xi(double E1sum, double sP0, double sP1, double sP2, double rn, double rnm1,
                                      double a0, double a1, double a2, double dt, double cell, double e1_const,
                                      double pscale) {
    const double E1 = cell * E1sum + e1_const;
    const double p1 = pscale * sP0, p2 = pscale * sP1, pp = pscale * sP2;
    const double S = sqrt(E1);
    const double rho = a1 * rn + a2 * rnm1;
    return (rho + (a0 * p2 - pp) / (2.0 * S)) / (a0 * (S - dt * p1 / (2.0 * S)));
}

// Close one step (one lane): copy the scalar block, then record the state X of the
// step (record sc.step_x: modified energy, mean, r) and the next state's xi, E_1,
// p1, S, and shift the r pair.  Reads fi.sc_in, writes fi.sc_out (already narrowed
// to one member).
__device__ inline void finish_step(const FinishIn& fi, double E1sum, const double (&sE)[NPART_E],
                                   const double (&sP)[NPART_P], double a0, double a1, double a2, double dt,
                                   const Geo& geo) {
    DevScalars s = *fi.sc_in;
    const double rn = s.r_n, rnm1 = s.r_nm1;
    const double E1 = geo.cell * E1sum + geo.e1_const;
    const double n0 = geo.pscale * sE[0], n1 = geo.pscale * sE[1];
    const double p1 = geo.pscale * sP[0], p2 = geo.pscale * sP[1], pp = geo.pscale * sP[2];
    const double S = sqrt(E1);
    const double xi = sav_xi(E1sum, sP[0], sP[1], sP[2], rn, rnm1, a0, a1, a2, dt, geo.cell, geo.e1_const,
                             geo.pscale);
    const double rnew = xi * S;
    const double energy = pair_energy(n0, n1, rn, rnm1, geo.pscale * sE[5], dt, geo);
    const double mean = sE[4] * geo.inv_npts;
    unsigned int fl = s.flags;
    if (!isfinite(E1) || !isfinite(p1) || !isfinite(p2) || !isfinite(pp) || !isfinite(xi) || !isfinite(energy))
        fl |= FLAG_NONFINITE;
    if (E1 < geo.volume * (1.0 - 1e-12)) fl |= FLAG_E1_BELOW_OMEGA;
    if (p1 > 0.0) fl |= FLAG_P1_POSITIVE;
    if (fi.check_rise && energy > s.energy_prev * (1.0 + fi.energy_tol)) fl |= FLAG_ENERGY_RISE;
    const long long step = s.step_x;
    Record* rc = fi.hist + (step % fi.hist_cap);
    rc->energy = energy;
    rc->mean = mean;
    rc->r = rn;
    Record* rn1 = fi.hist + ((step + 1) % fi.hist_cap);
    rn1->energy = 0.0;
    rn1->mean = 0.0;
    rn1->r = rnew;
    rn1->xi = xi;
    rn1->E1 = E1;
    rn1->p1 = p1;
    rn1->S = S;
    rn1->reserved = 0.0;
    s.xi = xi;
    s.r_nm1 = rn;
    s.r_n = rnew;
    s.energy_prev = energy;
    s.E1 = E1;
    s.p1 = p1;
    s.p2 = p2;
    s.ppsi = pp;
    s.S = S;
    s.mean = mean;
    s.flags = fl;
    s.last_record = step;
    s.step_x = step + 1;
    *fi.sc_out = s;
}

// FinishIn narrowed to member m of the batch.
__device__ inline FinishIn member_fin(const FinishIn& f, int m) {
    FinishIn r = f;
    r.partP = f.partP + (size_t)m * f.nPE * (f.nB > 0 ? NPART_P : NPART_PF);   // folded layout when nB = 0
    r.partE = f.partE + (size_t)m * f.nPE * NPART_E;
    r.partB = f.partB + (size_t)m * f.nB;
    r.sc_in = f.sc_in + m;
    r.sc_out = f.sc_out + m;
    r.hist = f.hist + (size_t)m * f.hist_cap;
    return r;
}

// What a pending update needs for xi, loaded before a kernel's own loads: the r
// pair and the xi a separate finish left, and (fin) the first sweep of the partial
// sums that give xi (E_1 partials, then the three inner-product partials).
struct XiInputs {
    PairSweep<1, NPART_P> first;
    double xi, rn, rnm1;
    __device__ inline void load(const FinishIn& fi, bool fin) {
        xi = fi.sc_in->xi;
        rn = fi.sc_in->r_n;
        rnm1 = fi.sc_in->r_nm1;
        if (fin) first.load(fi.partB, fi.nB, fi.partP, fi.nPE, threadIdx.x);
    }
    // wait for them here (PairSweep::settle)
    __device__ inline void settle(bool fin) {
        asm volatile("" : "+v"(xi), "+v"(rn), "+v"(rnm1));
        if (fin) first.settle();
    }
};

// Every workgroup of a launch reduces the previous step's partial sums in the
// same order and gets the same xi; workgroup 0 also closes the step (records,
// new scalar block).  All threads of the workgroup must call it.  `in` holds the
// r pair and the first sweep of the partials (XiInputs::load with fin).
__device__ inline double finish_in_kernel(const FinishIn& fi, const XiInputs& in, double a0, double a1, double a2,
                                          double dt, const Geo& geo) {
    double sBP[1 + NPART_P];
    block_sum_pair_from<1, NPART_P>(in.first, fi.partB, fi.nB, fi.partP, fi.nPE, sBP);
    const double xi = sav_xi(sBP[0], sBP[1], sBP[2], sBP[3], in.rn, in.rnm1, a0, a1, a2, dt, geo.cell,
                             geo.e1_const, geo.pscale);
    if (blockIdx.x == 0) {
        double sE[NPART_E];
        block_sum_partials<NPART_E>(fi.partE, fi.nPE, sE);
        if (threadIdx.x == 0) {
            const double sP[NPART_P] = {sBP[1], sBP[2], sBP[3]};
            finish_step(fi, sBP[0], sE, sP, a0, a1, a2, dt, geo);
        }
    }
    return xi;
}

__device__ inline double finish_in_kernel(const FinishIn& fi, double a0, double a1, double a2, double dt,
                                          const Geo& geo) {
    XiInputs in;
    in.load(fi, true);
    return finish_in_kernel(fi, in, a0, a1, a2, dt, geo);
}

// Store of transform results held in registers (element t + P m of each of C lines of
// the group) to outputs in which, for each element e, the workgroup's G lines are
// neighbours: through an LDS tile [c][e][g] (the line buffers, free once the transform is
// done) so that consecutive threads store consecutive lines, CH of the C lines per round
// (a round's tile, CH NL G entries, fits in the workgroup's G CH line buffers).
// The line index is swizzled by e when G is a power of two (bank spread).
// idx(c, e, gi) gives the element's position in output c, or a negative value for a line
// past the end.  All threads of the workgroup must call it.
template <typename T, typename PL, int C, int CH = C, class Idx>
__device__ inline void tiled_line_store(const cpx<T> (&v)[C][PL::E], cpx<T>* tile, int G, int g, int t,
                                        cpx<T>* const* out, size_t mbase, Idx idx) {
    constexpr int NL = PL::Nl, E = PL::E, P = PL::P;
    const int sw = (G & (G - 1)) == 0 ? G - 1 : 0;
    const int gi = threadIdx.x % G, step = blockDim.x / G;
#pragma unroll
    for (int c0 = 0; c0 < C; c0 += CH) {
        const int cn = C - c0 < CH ? C - c0 : CH;
        __syncthreads();   // the previous reads of the line buffers (transform or tile) are done
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (c < cn) {
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const int e = t + P * m;
                    tile[(c * NL + e) * G + (g ^ (e & sw))] = v[c0 + c][m];
                }
            }
        }
        __syncthreads();
        for (int ce = threadIdx.x / G; ce < cn * NL; ce += step) {
            const int c = ce / NL, e = ce - c * NL;
            const long long i = idx(c0 + c, e, gi);
            if (i >= 0) out[c0 + c][mbase + (size_t)i] = tile[(c * NL + e) * G + (gi ^ (e & sw))];
        }
    }
}

// ------------------------------------------------------------------ spectral inverse pass

// One group of P threads per spectral line.  Optional pending update
//   X = (udt xi (-|k|^2) N + ua1 C + ua2 P) / (ua0 + udt |k|^2 (a + |k|^4)),  Y = C
// (eq. scheme-SAV-1 solved for phi^{n+1}), else X = C, Y = P.  Partials of
// ||L^1/2 X||^2, ||L^1/2 (2X - Y)||^2, ||X||^2, ||Delta X||^2 (modified energy,
// eq. discrete energy; E_N, eq. energy-discrete-spectral).  Then the inverse
// transform along the line of phihat = e1 X + e2 Y and of i kappa1 phihat for the
// line's own axis.  The symbols of the other axes are constant along the line, so
// the later passes apply them (i kappa1_y before the y transform in 3-D, i kappa1_x
// as the real-space pass loads its rows): two fields out instead of d.
// FIN: the variant that can close the pending step itself (p.fin); without it the
// reduction's registers are not held (161 -> 106 VGPRs at 256 points, FP32), so a
// separately closed step runs more waves per SIMD.
// 3-D: the two lines of a group go through the exchanges and the output tile one at a
// time (one line buffer per group), so that workgroups of up to 512 threads (16 lines of
// 256 points) write runs of 16 neighbouring entries; 2-D keeps both lines at once.
template <typename T, int NL, int EE, int DIM, bool STAB, bool FIN>
__global__ void __launch_bounds__(DIM == 3 ? 512 : 256) k_spec_inv(SpecInvArgs<T> p) {
    using PL = Plan<NL, EE>;
    constexpr int E = PL::E, P = PL::P, C = 2, CH = DIM == 3 ? 1 : C;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* ltw = lds + p.G * CH * LdsLine<NL>::size;
    const int tid = threadIdx.x, g = tid / P, t = tid - g * P;
    const int line = xcd_block(blockIdx.x, gridDim.x) * p.G + g;
    const bool act = line < p.nlines;
    const int mem = blockIdx.y;
    const Geo geo = p.geos[mem];
    const size_t lbase = (size_t)mem * p.fs + (size_t)(act ? line : 0) * NL;
    const size_t mbase = (size_t)mem * p.fs;

    // all loads first (the update writes in place over `prev`, so later loads
    // must not wait behind earlier stores), the partial sums of xi before the
    // field values so that their reduction overlaps the field loads
    const FinishIn fi = member_fin(p.fi, mem);
    const bool fin = FIN && p.update && p.fin;
    XiInputs xin;
    if (p.update) xin.load(fi, fin);
    issue_barrier();
    // (lanes past the last line load line 0 of the member: finite values that reach
    // no output, their symbols being zero)
    cpx<T> cur[E], prv[E], nh[E];
    if (p.update) {
#pragma unroll
        for (int m = 0; m < E; ++m) nh[m] = p.nhat[lbase + t + P * m];
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const size_t i = lbase + t + P * m;
        cur[m] = p.cur[i];
        prv[m] = p.prev[i];
    }
    issue_barrier();
    double xi = 0.0;
    if (p.update) {
        xin.settle(fin);
        xi = fin ? finish_in_kernel(fi, xin, p.ua0, p.ua1, p.ua2, p.udt, geo) : xin.xi;
    }

    double acc[NPART_E] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    cpx<T> v[C][E];
    const T h1 = T(p.e1), h2 = T(p.e2);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int e = t + P * m;
        cpx<T> X = cur[m], Y = prv[m];
        int kx = 0, ky = 0, kz = 0;
        double k2 = 0.0, k1[3] = {0.0, 0.0, 0.0};
        if (act) {
            spec_index<DIM>(line, p.B, e, kx, ky, kz);
            spec_symbols<DIM>(geo, kx, ky, kz, k2, k1);
            if (p.update) {
                // in FP64 for both storage precisions: the k = 0 mode then keeps the mean
                // (Theorem 2.1) to the rounding of one store per step
                const double st = stab_sym<STAB>(geo, p.udt, k2);
                const double iA = 1.0 / (p.ua0 + p.udt * k2 * (geo.a + k2 * k2) + st);
                const double f1 = -p.udt * xi * k2 * iA, f2 = (p.ua1 + st) * iA, f3 = p.ua2 * iA;
                double xr = f1 * nh[m].x + f2 * cur[m].x + f3 * prv[m].x;
                double xi_ = f1 * nh[m].y + f2 * cur[m].y + f3 * prv[m].y;
                if (p.fhat) {   // forcing of the pending step (not written by this kernel)
                    const cpx<T> fh = p.fhat[lbase + e];
                    xr += p.udt * iA * (double)fh.x;
                    xi_ += p.udt * iA * (double)fh.y;
                }
                X = mk<T>(T(xr), T(xi_));
                Y = cur[m];
                p.out_new[lbase + e] = X;
            } else {
                pair_partials<T, STAB>(X, Y, kx, k2, line == 0 && e == 0, geo, acc);
            }
        }
        const cpx<T> ph = mk<T>(h1 * X.x + h2 * Y.x, h1 * X.y + h2 * Y.y);
        const T kk = T(k1[DIM - 1]);
        v[0][m] = ph;
        v[1][m] = mk<T>(-kk * ph.y, kk * ph.x);   // i kappa1 phihat along the line's axis
    }
    if (!p.update) store_energy_partials<STAB>(acc, p.part + NPART_E * ((size_t)mem * gridDim.x + blockIdx.x));
    if (p.want_grad) {
        stage_twiddles<T, PL>(ltw, p.tw, p.tws);
        fft_run<T, PL, +1, C, 0, CH>(v, lds + g * CH * LdsLine<NL>::size, t, ltw);
        if constexpr (DIM == 3) {
            // rotated output [e][lines]: the workgroup's lines are neighbours for each e
            const int line0 = xcd_block(blockIdx.x, gridDim.x) * p.G;
            tiled_line_store<T, PL, C, CH>(v, lds, p.G, g, t, p.out, mbase, [&](int, int e, int gi) -> long long {
                const int ln = line0 + gi;
                return ln < p.nlines ? (long long)e * p.nlines + ln : -1;
            });
        } else if (act) {
#pragma unroll
            for (int j = 0; j < C; ++j) {
                cpx<T>* o = p.out[j] + mbase;
#pragma unroll
                for (int m = 0; m < E; ++m) o[(size_t)(t + P * m) * p.nlines + line] = v[j][m];
            }
        }
    }
}

// ------------------------------------------------------------------ real-space pass

// Packing of real rows into complex lines.  The input fields are the rows of
// phihat (field 0, its x half spectrum; i kappa1_x times it is that of g_x), of g_y
// (field 1) and, in 3-D, of g_z (field 2).  2-D: one row per group, line 0 =
// g_x + i g_y.  3-D: two rows per group, lines (g_x + i g_y)(row 0),
// (g_x + i g_y)(row 1), g_z(row 0) + i g_z(row 1).  kx(c): the real part of line c
// is g_x, whose half row is i kappa1_x times the row of field 0.
//
// BETA (the quartic term (beta/4) phi^4 of the energy, phi itself needed in real space):
// two rows per group in both dimensions, and one more line, phi(row 0) + i phi(row 1)
// from the rows of field 0 as they are (last line: 2-D line 2, 3-D line 3); 2-D lines
// 0 and 1 are g_x + i g_y of rows 0 and 1.
template <int DIM, bool BETA = false>
struct RealPack {
    static constexpr int C = (DIM == 2 ? 1 : 3) + (BETA ? (DIM == 2 ? 2 : 1) : 0);
    static constexpr int RPG = (DIM == 2 && !BETA) ? 1 : 2;
    static constexpr int PHI = BETA ? C - 1 : -1;   // the line of phi
    __device__ static constexpr int fa(int c) { return c == PHI ? 0 : (DIM == 2 ? 0 : (c < 2 ? 0 : 2)); }
    __device__ static constexpr int fb(int c) { return c == PHI ? 0 : (DIM == 2 ? 1 : (c < 2 ? 1 : 2)); }
    __device__ static constexpr int ra(int c) { return c == PHI ? 0 : (c == 1 ? 1 : 0); }
    __device__ static constexpr int rb(int c) { return c == PHI ? 1 : (DIM == 2 ? (c == 1 ? 1 : 0) : (c == 0 ? 0 : 1)); }
    __device__ static constexpr bool kx(int c) { return c != PHI && fa(c) == 0; }
};

// i kappa1_x(k) z and -i kappa1_x(k) z for x wavenumber k <= N/2 (the odd-order symbol
// drops Nyquist)
template <typename T>
__device__ inline cpx<T> mul_ikx(cpx<T> z, int k, int n, double k0) {
    const T kk = T(sym1(k, n, k0));
    return mk<T>(-kk * z.y, kk * z.x);
}
template <typename T>
__device__ inline cpx<T> mul_mikx(cpx<T> z, int k, int n, double k0) {
    const T kk = T(sym1(k, n, k0));
    return mk<T>(kk * z.y, -kk * z.x);
}

// Load element e (0..N-1) of the complex line whose real part is the real row
// with half spectrum H1 and whose imaginary part has half spectrum H2:
// W(e) = H1(e) + i H2(e), H(e) = conj(H(N - e)) above N/2; the self-conjugate
// bins 0 and N/2 keep their real parts only.  H2 = h2; H1 = h1, or with KX
// H1 = i kappa1_x h1 (symbol k0).
template <typename T, int N, bool KX>
__device__ inline cpx<T> load_packed(const cpx<T>* h1, const cpx<T>* h2, int e, double k0) {
    cpx<T> a, b;
    const int k = 2 * e <= N ? e : N - e;
    a = h1[k];
    b = h2[k];
    if constexpr (KX) a = mul_ikx(a, k, N, k0);
    if (2 * e <= N) {
        if (e == 0 || 2 * e == N) {
            a.y = T(0);
            b.y = T(0);
        }
    } else {
        a = conj(a);
        b = conj(b);
    }
    return mk<T>(a.x - b.y, a.y + b.x);
}

// Value v of lane src of the wave (ds_bpermute on its 32-bit words).
template <typename T>
__device__ inline cpx<T> lane_fetch(cpx<T> v, int src) {
    constexpr int W = (int)(sizeof(cpx<T>) / 4);
    union U {
        cpx<T> c;
        int w[W];
    } u;
    u.c = v;
#pragma unroll
    for (int i = 0; i < W; ++i) u.w[i] = __builtin_amdgcn_ds_bpermute(src << 2, u.w[i]);
    return u.c;
}

// The complex line W = H1 + i H2 of two real rows with half spectra h1, h2, element
// t + P m in w[m], as load_packed gives it, but each half-spectrum entry is loaded once:
// thread t loads the entries e = t + P m with m < E/2 (all lanes also read the
// self-conjugate bin N/2, which thread 0 keeps), and an element e > N/2, whose value
// W(e) = conj H1(N - e) + i conj H2(N - e) comes from entry N - e, is formed by the lane
// that loaded N - e and moved across lanes: element m >= E/2 of thread t > 0 mirrors
// element E - 1 - m of thread P - t, and thread 0's mirror its own element E - m.
// Needs the P threads of a line within one wave (P <= 64).  In two halves, so that a
// kernel issues the loads of all its lines before the first exchange waits for any of
// them: packed_fetch (the loads) and packed_mirror (all P lanes must call it; with KX,
// H1 = i kappa1_x h1, whose Nyquist bin is zero).
template <typename T, typename PL>
struct PackedRaw {
    cpx<T> a[PL::E / 2], b[PL::E / 2], an, bn;
};

template <typename T, typename PL>
__device__ inline void packed_fetch(const cpx<T>* h1, const cpx<T>* h2, int t, PackedRaw<T, PL>& r) {
    constexpr int H = PL::E / 2, P = PL::P, N = PL::Nl;
    static_assert(P <= 64, "a line must lie within one wave");
#pragma unroll
    for (int m = 0; m < H; ++m) {
        r.a[m] = h1[t + P * m];
        r.b[m] = h2[t + P * m];
    }
    r.an = h1[N / 2];
    r.bn = h2[N / 2];
}

template <typename T, typename PL, bool KX>
__device__ inline void packed_mirror(PackedRaw<T, PL>& r, int t, cpx<T> (&w)[PL::E], double k0) {
    constexpr int E = PL::E, P = PL::P, N = PL::Nl, H = E / 2;
    cpx<T>* a = r.a;
    cpx<T>* b = r.b;
    if constexpr (KX) {
#pragma unroll
        for (int m = 0; m < H; ++m) a[m] = mul_ikx(a[m], t + P * m, N, k0);
        r.an = mk<T>(T(0), T(0));
    }
    if (t == 0) {
        a[0].y = T(0);
        b[0].y = T(0);
    }
    cpx<T> mv[H];   // what this lane's entries give the mirrored elements: conj H1 + i conj H2
#pragma unroll
    for (int m = 0; m < H; ++m) {
        w[m] = mk<T>(a[m].x - b[m].y, a[m].y + b[m].x);
        mv[m] = mk<T>(a[m].x + b[m].y, b[m].x - a[m].y);
    }
    const int lane = (int)(threadIdx.x & 63);
    const int src = lane - t + ((P - t) & (P - 1));
#pragma unroll
    for (int m = H; m < E; ++m) {
        const cpx<T> x = lane_fetch(mv[E - 1 - m], src);
        if (t != 0) w[m] = x;
        else w[m] = m == H ? mk<T>(r.an.x, r.bn.x) : mv[E - m];
    }
}

// packed_fetch + packed_mirror for lines that span several waves (P > 64): the entries each thread
// loads (t + P m for m < E/2, and the self-conjugate bin N/2) are staged in the group's line
// buffer, stage[0 .. N/2] (H1, with KX times i kappa1_x) and stage[N/2 + 1 .. N + 1] (H2),
// and each thread reads the entries N - e of its mirrored elements from there.  The buffer
// must hold N + 2 entries and be free; all threads of the workgroup must call it (barrier).
// The next write to the buffer must follow a barrier (fft_run's second pass has one).
template <typename T, typename PL, bool KX>
__device__ inline void load_packed_staged(const cpx<T>* h1, const cpx<T>* h2, int t, cpx<T> (&w)[PL::E], double k0,
                                          cpx<T>* stage, bool act) {
    constexpr int E = PL::E, P = PL::P, N = PL::Nl, H = E / 2, NXH = N / 2 + 1;
    static_assert(N + 2 <= LdsLine<N>::size, "staging needs N + 2 entries of the line buffer");
#pragma unroll
    for (int m = 0; m < H; ++m) {
        const int e = t + P * m;
        cpx<T> a = h1[e], b = h2[e];
        if constexpr (KX) a = mul_ikx(a, e, N, k0);
        if (e == 0) {
            a.y = T(0);
            b.y = T(0);
        }
        stage[e] = a;
        stage[NXH + e] = b;
        w[m] = mk<T>(a.x - b.y, a.y + b.x);
    }
    if (t == 0) {
        cpx<T> a = h1[N / 2], b = h2[N / 2];
        stage[N / 2] = KX ? mk<T>(T(0), T(0)) : mk<T>(a.x, T(0));
        stage[NXH + N / 2] = mk<T>(b.x, T(0));
    }
    __syncthreads();
#pragma unroll
    for (int m = H; m < E; ++m) {
        const int e = t + P * m, k = N - e;   // e >= N/2; k = N/2 only for t = 0, m = H
        const cpx<T> a = stage[k], b = stage[NXH + k];
        w[m] = e == N / 2 ? mk<T>(a.x, b.x) : mk<T>(a.x + b.y, b.x - a.y);   // conj H1 + i conj H2
    }
    if (!act) {
#pragma unroll
        for (int m = 0; m < E; ++m) w[m] = mk<T>(T(0), T(0));
    }
}

// Two neighbouring complex values in one store (dst aligned to twice the element).
template <typename T>
__device__ inline void store_pair(cpx<T>* dst, cpx<T> a, cpx<T> b) {
    struct alignas(2 * sizeof(cpx<T>)) Pair {
        cpx<T> a, b;
    };
    *reinterpret_cast<Pair*>(dst) = Pair{a, b};
}

// Gradient rows (half spectra along x) -> C2R -> s = |grad phihat|^2,
// E_1 partial sum (c4/4) s^2 - s, q = c4 s grad phihat (eq. nonlinear chem pot-1) ->
// R2C -> flux spectra written rotated [kx][rows]: -i kappa1_x Q_x (the x term of the
// divergence in N, applied here where kx is known), Q_y and (3-D) Q_z.  FWD = false:
// E_1 only.
// BETA: the rows of phi come along (RealPack), the E_1 partial gains (beta/4) phi^4 and
// the x field written is -i kappa1_x Q_x + F(beta phi^3), i.e. N gains beta phi^3.
template <typename T, int NX, int EE, int DIM, bool FWD, bool BETA>
__global__ void __launch_bounds__(256) k_real_pass(RealArgs<T> p) {
    using PK = RealPack<DIM, BETA>;
    using PL = Plan<NX, EE>;
    constexpr int E = PL::E, P = PL::P, C = PK::C, RPG = PK::RPG;
    constexpr int NXH = NX / 2 + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw) + (threadIdx.x / P) * C * LdsLine<NX>::size;
    cpx<T>* ltw = reinterpret_cast<cpx<T>*>(smem_raw) + p.G * C * LdsLine<NX>::size;
    const int tid = threadIdx.x, g = tid / P, t = tid - g * P;
    const int row0 = (xcd_block(blockIdx.x, gridDim.x) * p.G + g) * RPG;
    const bool act = row0 < p.nrows;
    const int mem = blockIdx.y;
    const Geo geo = p.geos[mem];
    const size_t mbase = (size_t)mem * p.fs;

    // twiddle loads first, so that the wait for them before their LDS store does not
    // include the field loads
    TwStage<T, PL> tws;
    tws.load(p.tw, p.tws);
    issue_barrier();
    cpx<T> v[C][E];
    if constexpr (P <= 64) {
        // every line's loads first, then the exchanges (c is a constant once the loops
        // are unrolled)
        PackedRaw<T, PL> raw[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const cpx<T>* h1 = p.in[PK::fa(c)] + mbase + (size_t)(act ? row0 + PK::ra(c) : 0) * NXH;
            const cpx<T>* h2 = p.in[PK::fb(c)] + mbase + (size_t)(act ? row0 + PK::rb(c) : 0) * NXH;
            packed_fetch<T, PL>(h1, h2, t, raw[c]);
        }
        issue_barrier();
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (PK::kx(c)) packed_mirror<T, PL, true>(raw[c], t, v[c], geo.k0x);
            else packed_mirror<T, PL, false>(raw[c], t, v[c], 0.0);
            if (!act) {
#pragma unroll
                for (int m = 0; m < E; ++m) v[c][m] = mk<T>(0, 0);
            }
        }
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const cpx<T>* h1 = p.in[PK::fa(c)] + mbase + (size_t)(act ? row0 + PK::ra(c) : 0) * NXH;
            const cpx<T>* h2 = p.in[PK::fb(c)] + mbase + (size_t)(act ? row0 + PK::rb(c) : 0) * NXH;
            // the group's line buffer c is free until the transform
            cpx<T>* stage = lds + c * LdsLine<NX>::size;
            if (PK::kx(c)) load_packed_staged<T, PL, true>(h1, h2, t, v[c], geo.k0x, stage, act);
            else load_packed_staged<T, PL, false>(h1, h2, t, v[c], 0.0, stage, act);
        }
    }
    issue_barrier();
    tws.store(ltw);
    fft_run<T, PL, +1, C>(v, lds, t, ltw);

    const T sc = T(geo.inv_npts), c4 = T(geo.c4), bt = T(geo.beta);
    const double qc4 = 0.25 * geo.c4, qb4 = 0.25 * geo.beta;
    double acc[1] = {0.0};
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if constexpr (BETA) {
            // phi of the two rows: P = beta phi^3, E_1 density (beta/4) phi^4
            const T f0 = v[PK::PHI][m].x * sc, f1 = v[PK::PHI][m].y * sc;
            const T f02 = f0 * f0, f12 = f1 * f1;
            acc[0] += qb4 * ((double)f02 * (double)f02 + (double)f12 * (double)f12);
            v[PK::PHI][m] = mk<T>(bt * f02 * f0, bt * f12 * f1);
        }
        if constexpr (DIM == 2 && BETA) {
            const T ax = v[0][m].x * sc, ay = v[0][m].y * sc, bx = v[1][m].x * sc, by = v[1][m].y * sc;
            const T sa = ax * ax + ay * ay, sb = bx * bx + by * by;
            acc[0] += qc4 * (double)sa * (double)sa - (double)sa + qc4 * (double)sb * (double)sb - (double)sb;
            const T qa = c4 * sa, qb = c4 * sb;
            v[0][m] = mk<T>(qa * ax, qa * ay);
            v[1][m] = mk<T>(qb * bx, qb * by);
        } else if constexpr (DIM == 2) {
            const T gx = v[0][m].x * sc, gy = v[0][m].y * sc;
            const T s = gx * gx + gy * gy;
            acc[0] += qc4 * (double)s * (double)s - (double)s;
            const T q = c4 * s;
            v[0][m] = mk<T>(q * gx, q * gy);
        } else {
            const T ax = v[0][m].x * sc, ay = v[0][m].y * sc, az = v[2][m].x * sc;
            const T bx = v[1][m].x * sc, by = v[1][m].y * sc, bz = v[2][m].y * sc;
            const T sa = ax * ax + ay * ay + az * az;
            const T sb = bx * bx + by * by + bz * bz;
            acc[0] += qc4 * (double)sa * (double)sa - (double)sa + qc4 * (double)sb * (double)sb - (double)sb;
            const T qa = c4 * sa, qb = c4 * sb;
            v[0][m] = mk<T>(qa * ax, qa * ay);
            v[1][m] = mk<T>(qb * bx, qb * by);
            v[2][m] = mk<T>(qa * az, qb * bz);
        }
    }
    if (!act) acc[0] = 0.0;

    if constexpr (FWD) {
        fft_run<T, PL, -1, C>(v, lds, t, ltw);
        // split V = Q1 + i Q2 into the two half spectra: Q1(k) = (V(k) + conj V(-k)) / 2,
        // Q2(k) = (V(k) - conj V(-k)) / (2 i).
        __syncthreads();
        const T half = T(0.5);
        if constexpr (DIM == 3 && NX >= 32 && E <= 8) {
            // (4 or 8 values per thread; at 256^3 the run length decides: 2G rows of 8-byte
            // values per wavenumber, 64 bytes at 4 values and 256 threads, 128 bytes at 8,
            // 94.5 against 104.3 us; 16 per thread keeps the per-thread pair stores below.)
            // Rotated output through an LDS tile, so that each wave writes whole lines: the
            // workgroup's 2G rows are neighbours in every output, [k][rows].  The lines go
            // line-major across the groups (line c of group g at (c G + g) LS); then one
            // field at a time (g_z first, which frees line 2's region for the tile, then
            // g_x and g_y): its values for the group's two rows into registers, the tile
            // (pair index swizzled by k when G is a power of two, to spread the banks), and
            // consecutive threads store consecutive row pairs.  The tile, (NX/2 + 1) x 2G
            // entries, fits in line 2's region (G LS entries) for NX >= 32.
            constexpr int LS = LdsLine<NX>::size, NK = E / 2 + 1;
            cpx<T>* const lb = reinterpret_cast<cpx<T>*>(smem_raw);
            const int G = p.G, R2 = 2 * G, sw = (G & (G - 1)) == 0 ? G - 1 : 0;
            const int row_base = xcd_block(blockIdx.x, gridDim.x) * G * RPG;
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int m = 0; m < E; ++m) lb[(c * G + g) * LS + lds_pad<NX>(t + P * m)] = v[c][m];
            __syncthreads();
            auto split = [&](int c, int k, cpx<T>& q1, cpx<T>& q2) {
                const cpx<T> Vk = lb[(c * G + g) * LS + lds_pad<NX>(k)];
                const cpx<T> Vm = lb[(c * G + g) * LS + lds_pad<NX>((NX - k) & (NX - 1))];
                q1 = mk<T>(half * (Vk.x + Vm.x), half * (Vk.y - Vm.y));
                q2 = mk<T>(half * (Vk.y + Vm.y), half * (Vm.x - Vk.x));
            };
            cpx<T>* const tile = lb + 2 * G * LS;
            const int st_k0 = threadIdx.x / G, st_j = threadIdx.x - st_k0 * G;
            const int st_row = row_base + RPG * st_j;
            const bool st_ok = st_row < p.nrows;
            const size_t st_off = mbase + (size_t)st_k0 * p.nrows + st_row, st_step = (size_t)P * p.nrows;
#pragma unroll
            for (int f0 = 0; f0 < 3; ++f0) {
                const int f = f0 == 0 ? 2 : f0 - 1;
                cpx<T> ra[NK], rb[NK];   // field f at rows 2g, 2g + 1 and k = t + P m
#pragma unroll
                for (int m = 0; m < NK; ++m) {
                    const int k = m < E / 2 ? t + P * m : NX / 2;   // the last: t = 0 only
                    cpx<T> x, y;
                    if (f == 2) {
                        split(2, k, ra[m], rb[m]);
                    } else if (f == 0) {
                        split(0, k, ra[m], x);
                        split(1, k, rb[m], y);
                        ra[m] = mul_mikx(ra[m], k, NX, geo.k0x);
                        rb[m] = mul_mikx(rb[m], k, NX, geo.k0x);
                        if constexpr (BETA) {   // + F(beta phi^3) of the two rows
                            cpx<T> pa, pb;
                            split(PK::PHI, k, pa, pb);
                            ra[m] = ra[m] + pa;
                            rb[m] = rb[m] + pb;
                        }
                    } else {
                        split(0, k, x, ra[m]);
                        split(1, k, y, rb[m]);
                    }
                }
                __syncthreads();   // the reads of the tile region (line 2, the previous tile) are done
#pragma unroll
                for (int m = 0; m < NK; ++m) {
                    if (m == E / 2 && t != 0) break;
                    const int k = t + P * m, jj = g ^ (k & sw);
                    tile[k * R2 + 2 * jj] = ra[m];
                    tile[k * R2 + 2 * jj + 1] = rb[m];
                }
                __syncthreads();
                // the workgroup is G P threads: thread (k0, j) stores pair j of wavenumbers
                // k0, k0 + P, ... (no division in the loop)
                if (st_ok) {
                    cpx<T>* dst = p.out[f] + st_off;
                    for (int k = st_k0; k < NXH; k += P, dst += st_step) {
                        const int jj = st_j ^ (k & sw);
                        store_pair(dst, tile[k * R2 + 2 * jj], tile[k * R2 + 2 * jj + 1]);
                    }
                }
            }
        } else {
            line_store<T, PL, C>(v, lds, t);
            __syncthreads();
            if (act) {
                auto split = [&](int c, int k, cpx<T>& q1, cpx<T>& q2) {
                    const cpx<T> Vk = lds[c * LdsLine<NX>::size + lds_pad<NX>(k)];
                    const cpx<T> Vm = lds[c * LdsLine<NX>::size + lds_pad<NX>((NX - k) & (NX - 1))];
                    q1 = mk<T>(half * (Vk.x + Vm.x), half * (Vk.y - Vm.y));
                    q2 = mk<T>(half * (Vk.y + Vm.y), half * (Vm.x - Vk.x));
                };
                if constexpr (DIM == 3) {
                    // the group's two rows are neighbours in every output: one store of the
                    // pair (rows row0, row0 + 1; row0 is even) per field and wavenumber
#pragma unroll
                    for (int m = 0; m <= E / 2; ++m) {
                        const int k = t + P * m;
                        if (m == E / 2 && t != 0) break;
                        cpx<T> q1[C], q2[C];
#pragma unroll
                        for (int c = 0; c < C; ++c) split(c, k, q1[c], q2[c]);
                        const size_t o = mbase + (size_t)k * p.nrows + row0;
                        cpx<T> r0 = mul_mikx(q1[0], k, NX, geo.k0x), r1 = mul_mikx(q1[1], k, NX, geo.k0x);
                        if constexpr (BETA) {
                            r0 = r0 + q1[PK::PHI];
                            r1 = r1 + q2[PK::PHI];
                        }
                        store_pair(p.out[0] + o, r0, r1);         // lines 0, 1: g_x of rows 0, 1
                        store_pair(p.out[1] + o, q2[0], q2[1]);   // g_y of rows 0, 1
                        store_pair(p.out[2] + o, q1[2], q2[2]);   // line 2: g_z of rows 0, 1
                    }
                } else if constexpr (BETA) {
                    // 2-D with phi: rows row0, row0 + 1 (even row0) are neighbours in both outputs
#pragma unroll
                    for (int m = 0; m <= E / 2; ++m) {
                        const int k = t + P * m;
                        if (m == E / 2 && t != 0) break;
                        cpx<T> q1[C], q2[C];
#pragma unroll
                        for (int c = 0; c < C; ++c) split(c, k, q1[c], q2[c]);
                        const size_t o = mbase + (size_t)k * p.nrows + row0;
                        store_pair(p.out[0] + o, mul_mikx(q1[0], k, NX, geo.k0x) + q1[PK::PHI],
                                   mul_mikx(q1[1], k, NX, geo.k0x) + q2[PK::PHI]);
                        store_pair(p.out[1] + o, q2[0], q2[1]);
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        cpx<T>* o1 = p.out[PK::fa(c)] + mbase;
                        cpx<T>* o2 = p.out[PK::fb(c)] + mbase;
                        const int r1 = row0 + PK::ra(c), r2 = row0 + PK::rb(c);
#pragma unroll
                        for (int m = 0; m <= E / 2; ++m) {
                            const int k = t + P * m;
                            if (m == E / 2 && t != 0) break;
                            cpx<T> q1, q2;
                            split(c, k, q1, q2);
                            if (PK::kx(c)) q1 = mul_mikx(q1, k, NX, geo.k0x);
                            o1[(size_t)k * p.nrows + r1] = q1;
                            o2[(size_t)k * p.nrows + r2] = q2;
                        }
                    }
                }
            }
        }
    }
    block_sum_store<1>(acc, p.part + (size_t)mem * gridDim.x + blockIdx.x);
}

// ------------------------------------------------------------------ generic line pass

template <typename T, int NL, int EE, int DIR, int OMODE, int C>
__global__ void __launch_bounds__(256) k_pass(PassArgs<T> p) {
    using PL = Plan<NL, EE>;
    constexpr int E = PL::E, P = PL::P;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* ltw = lds + p.G * C * LdsLine<NL>::size;
    const int tid = threadIdx.x, g = tid / P, t = tid - g * P;
    const int line = xcd_block(blockIdx.x, gridDim.x) * p.G + g;
    const bool act = line < p.nlines;
    const size_t mbase = (size_t)blockIdx.y * p.fs;
    const size_t lbase = (size_t)(act ? line : 0) * NL;
    cpx<T> v[C][E];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int m = 0; m < E; ++m) v[c][m] = act ? p.in[c][mbase + lbase + t + P * m] : mk<T>(0, 0);
    stage_twiddles<T, PL>(ltw, p.tw, p.tws);
    fft_run<T, PL, DIR, C>(v, lds + g * C * LdsLine<NL>::size, t, ltw);
    if (!act) return;
    const int a = line / p.B, b = line - a * p.B;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        cpx<T>* o = p.out[c] + mbase;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int e = t + P * m;
            size_t idx;
            if constexpr (OMODE == OUT_KEEP) idx = lbase + e;
            else if constexpr (OMODE == OUT_SWAP) idx = ((size_t)a * NL + e) * p.B + b;
            else idx = (size_t)e * p.nlines + line;
            o[idx] = v[c][m];
        }
    }
}

// ------------------------------------------------------------------ 3-D y passes of a step

// Lines along y, [a][b][Y] with b the faster line index (inverse: a = z, b = kx;
// forward: a = kx, b = z), written [a][Y][b] through the LDS tile.
// Inverse (DIR = +1): in[0] = Psi, in[1] = Psi_z, the z transforms of phihat and of
// i kappa1_z phihat; out[0..2] = the y transforms of Psi (i kappa1_x times it is the
// x half spectrum of g_x, applied by the real-space pass), of i kappa1_y Psi (g_y) and
// of Psi_z (g_z).  Forward (DIR = -1): in[0..2] = -i kappa1_x Q_x, Q_y, Q_z after the
// x transform; out[0] = V0 - i kappa1_y V1 and out[1] = V2 of their y transforms V0..V2,
// so that only the z term of the divergence is left for the last pass.
// The three lines of a group go through the transform's exchanges and the output tile
// one at a time (YPASS_CH line buffers per group), so that a workgroup of up to 512
// threads holds 16 lines of 256 points in 35 KB of LDS and writes runs of 16 neighbouring
// entries (128 bytes in FP32): 256^3 y passes 89 -> 82 and 82 -> 75 us inside the step,
// against 8 lines with all three lines exchanged at once.
template <typename T, int NL, int EE, int DIR>
__global__ void __launch_bounds__(512) k_ypass(PassArgs<T> p) {
    using PL = Plan<NL, EE>;
    constexpr int E = PL::E, P = PL::P, C = 3, CH = YPASS_CH;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* ltw = lds + p.G * CH * LdsLine<NL>::size;
    const int tid = threadIdx.x, g = tid / P, t = tid - g * P;
    const int line = xcd_block(blockIdx.x, gridDim.x) * p.G + g;
    const bool act = line < p.nlines;
    const int mem = blockIdx.y;
    const Geo geo = p.geos[mem];
    const size_t mbase = (size_t)mem * p.fs;
    const size_t lbase = mbase + (size_t)(act ? line : 0) * NL;
    TwStage<T, PL> tws;
    tws.load(p.tw, p.tws);
    issue_barrier();
    cpx<T> v[C][E];
    if constexpr (DIR > 0) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int e = t + P * m;
            const cpx<T> a = p.in[0][lbase + e], b = p.in[1][lbase + e];
            const T ky = T(sym1(e, geo.ny, geo.k0y));
            v[0][m] = a;
            v[1][m] = mk<T>(-ky * a.y, ky * a.x);   // i kappa1_y Psi
            v[2][m] = b;
        }
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int m = 0; m < E; ++m) v[c][m] = p.in[c][lbase + t + P * m];
    }
    // (lanes past the last line loaded line 0 of the member; they store nothing)
    issue_barrier();
    tws.store(ltw);
    fft_run<T, PL, DIR, C, 0, CH>(v, lds + g * CH * LdsLine<NL>::size, t, ltw);
    const int line0 = xcd_block(blockIdx.x, gridDim.x) * p.G;
    auto idx = [&](int, int e, int gi) -> long long {
        const int ln = line0 + gi;
        if (ln >= p.nlines) return -1;
        const int a = ln / p.B, b = ln - a * p.B;
        return ((long long)a * NL + e) * p.B + b;
    };
    if constexpr (DIR > 0) {
        tiled_line_store<T, PL, 3, CH>(v, lds, p.G, g, t, p.out, mbase, idx);
    } else {
        cpx<T> w[2][E];
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const T ky = T(sym1(t + P * m, geo.ny, geo.k0y));
            w[0][m] = mk<T>(v[0][m].x + ky * v[1][m].y, v[0][m].y - ky * v[1][m].x);   // V0 - i kappa1_y V1
            w[1][m] = v[2][m];
        }
        tiled_line_store<T, PL, 2, CH < 2 ? CH : 2>(w, lds, p.G, g, t, p.out, mbase, idx);
    }
}

// ------------------------------------------------------------------ spectral forward pass + solve

// Forward transform along the last axis of the two flux fields the earlier passes
// leave: V0, in which every divergence term but the last axis's is already applied
// (2-D: -i kappa1_x Q_x; 3-D: -i kappa1_x Q_x - i kappa1_y Q_y), and V1 = Q of the last
// axis.  Then N = V0 - i kappa1 V1 - 2 |k|^2 phihat (eq. nonlinear chem pot-1, divergence
// and the Laplacian part of N), the two solves and the inner products.  In terms of
// xi = r^{n+1} / sqrt(E_1): with phi^{n+1} = dt xi b1 + b2, b1 = A^-1 Delta N,
// b2 = A^-1 psi, the r equation (eq. scheme-SAV-1, second line) gives
//   xi = [rho + (a0 p2 - p_psi) / (2S)] / [a0 (S - dt p1 / (2S))],
// p1 = <N, b1> <= 0 (eq. solver-5), p2 = <N, b2>, p_psi = <N, psi>, S = sqrt(E_1); this
// kernel forms the partial sums of p1, p2 and p_psi.
// Stabilized scheme: A gains stab dt^2 |k|^4 and b2 = A^-1 (psi + stab dt^2 |k|^4 phi^n);
// the r equation, and so p_psi, keeps psi.
// FOLD (the step is closed by a separate kernel): each workgroup also adds its slice of the
// real-space pass's E_1 partials and stores NPART_PF partials (else NPART_P).
template <typename T, int NL, int EE, int DIM, int MODE, bool STAB, bool FOLD>
__global__ void __launch_bounds__(256) k_spec_fwd(SpecFwdArgs<T> p) {
    using PL = Plan<NL, EE>;
    constexpr int E = PL::E, P = PL::P, C = 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* ltw = lds + p.G * C * LdsLine<NL>::size;
    const int tid = threadIdx.x, g = tid / P, t = tid - g * P;
    const int line = xcd_block(blockIdx.x, gridDim.x) * p.G + g;
    const bool act = line < p.nlines;
    const int mem = blockIdx.y;
    const Geo geo = p.geos[mem];
    const size_t lbase = (size_t)mem * p.fs + (size_t)(act ? line : 0) * NL;

    // The flux lines, then the pair (X, Y), which is needed only after the transform.
    // 3-D: the pair's loads are issued before the transform and are in flight while it
    // runs (lanes past the last line load line 0 of the member; nothing of theirs
    // reaches an output).  2-D: after it; there the early loads compete with the flux
    // loads the transform waits for and the step is slower (measured on 1024^2).
    // this workgroup's fixed slice [bj0, bj1) of the real-space pass's E_1 partials: the
    // first entry of each thread loaded ahead of everything (branch free: an index past the
    // slice reads entry 0 and adds nothing), so that waiting for the field loads covers it
    int bj = 0, bj1 = 0;
    double bval = 0.0;
    if constexpr (MODE != FWD_GHOST && FOLD) {
        const int bj0 = (int)((long long)p.nB * blockIdx.x / gridDim.x);
        bj1 = (int)((long long)p.nB * (blockIdx.x + 1) / gridDim.x);
        bj = bj0 + (int)threadIdx.x;
        bval = p.partB[(size_t)mem * p.nB + (bj < bj1 ? bj : 0)];
        issue_barrier();
    }
    cpx<T> v[C][E], Xs[E], Ys[E];
    auto load_pair = [&](bool all) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            Xs[m] = (all || act) ? p.X[lbase + t + P * m] : mk<T>(0, 0);
            Ys[m] = (all || act) ? p.Y[lbase + t + P * m] : mk<T>(0, 0);
        }
    };
#pragma unroll
    for (int j = 0; j < C; ++j)
#pragma unroll
        for (int m = 0; m < E; ++m)
            v[j][m] = (DIM == 3 || act) ? p.in[j][lbase + t + P * m] : mk<T>(0, 0);
    stage_twiddles<T, PL>(ltw, p.tw, p.tws);
    if constexpr (DIM == 3) {
        load_pair(true);
        issue_barrier();
    }
    fft_run<T, PL, -1, C>(v, lds + g * C * LdsLine<NL>::size, t, ltw);
    if constexpr (DIM == 2) load_pair(false);

    double acc[NPART_PF] = {0.0, 0.0, 0.0, 0.0};
    double accE[NPART_E] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (MODE != FWD_GHOST && FOLD) {
        // the rest of this workgroup's slice of the real-space partials (when it is longer
        // than the workgroup), then the entries loaded first
        for (int j = bj + (int)blockDim.x; j < bj1; j += (int)blockDim.x) acc[3] += p.partB[(size_t)mem * p.nB + j];
        acc[3] += bj < bj1 ? bval : 0.0;
    }
    if (act) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int e = t + P * m;
            int kx, ky, kz;
            double k2, k1[3];
            spec_index<DIM>(line, p.B, e, kx, ky, kz);
            spec_symbols<DIM>(geo, kx, ky, kz, k2, k1);
            const cpx<T> X = Xs[m], Y = Ys[m];
            const double phx = p.e1 * X.x + p.e2 * Y.x, phy = p.e1 * X.y + p.e2 * Y.y;
            // N = V0 - i kappa1 V1 - 2 |k|^2 phihat (kappa1 of the line's axis)
            const double kl = k1[DIM - 1];
            const double Nx = (double)v[0][m].x + kl * (double)v[1][m].y - 2.0 * k2 * phx;
            const double Ny = (double)v[0][m].y - kl * (double)v[1][m].x - 2.0 * k2 * phy;
            if constexpr (MODE != FWD_GHOST) {
                const double psx = p.a1 * X.x + p.a2 * Y.x, psy = p.a1 * X.y + p.a2 * Y.y;
                const double st = stab_sym<STAB>(geo, p.dt, k2);
                const double iA = 1.0 / (p.a0 + p.dt * k2 * (geo.a + k2 * k2) + st);
                const double w = hweight(kx, geo.nx);
                const double re = Nx * psx + Ny * psy;
                acc[0] -= w * k2 * (Nx * Nx + Ny * Ny) * iA;
                if constexpr (STAB) acc[1] += w * (re + st * (Nx * X.x + Ny * X.y)) * iA;
                else acc[1] += w * re * iA;
                if constexpr (MODE == FWD_SOLVE_FORCED) {   // b2 = A^{-1} (psi + dt f): <N, b2> gains dt <N, A^{-1} f>
                    const cpx<T> f = p.fhat[lbase + e];
                    acc[1] += w * p.dt * (Nx * (double)f.x + Ny * (double)f.y) * iA;
                }
                acc[2] += w * re;
                pair_partials<T, STAB>(X, Y, kx, k2, line == 0 && e == 0, geo, accE);
                p.nhat[lbase + e] = mk<T>(T(Nx), T(Ny));
            } else {
                // phi^{-1} = phi^0 - dt Delta_N (N + L_N phi^0)  (eq. scheme-SAV-initial-1)
                const double Lk = geo.a + k2 * k2;
                p.ghost_out[lbase + e] = mk<T>(T(X.x + p.dt * k2 * (Nx + Lk * X.x)), T(X.y + p.dt * k2 * (Ny + Lk * X.y)));
            }
        }
    }
    if constexpr (MODE != FWD_GHOST) {
        const size_t wg = (size_t)mem * gridDim.x + blockIdx.x;
        if constexpr (FOLD) {
            block_sum_store<NPART_PF>(acc, p.partP + NPART_PF * wg);
        } else {
            double a3[NPART_P] = {acc[0], acc[1], acc[2]};
            block_sum_store<NPART_P>(a3, p.partP + NPART_P * wg);
        }
        store_energy_partials<STAB>(accE, p.partE + NPART_E * wg);
    }
}

// ------------------------------------------------------------------ elementwise pending update

template <typename T, int DIM, bool STAB>
__global__ void __launch_bounds__(256) k_update(UpdateArgs<T> p) {
    const int mem = blockIdx.y;
    const Geo geo = p.geos[mem];
    const FinishIn fi = member_fin(p.fi, mem);
    const double xi = p.fin ? finish_in_kernel(fi, p.ua0, p.ua1, p.ua2, p.udt, geo) : fi.sc_in->xi;
    const size_t mbase = (size_t)mem * p.fs;
    double acc[NPART_E] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < p.total;
         i += (long long)gridDim.x * blockDim.x) {
        const int line = (int)(i / p.NL), e = (int)(i - (long long)line * p.NL);
        int kx, ky, kz;
        double k2, k1[3];
        spec_index<DIM>(line, p.B, e, kx, ky, kz);
        spec_symbols<DIM>(geo, kx, ky, kz, k2, k1);
        const cpx<T> cur = p.cur[mbase + i], prv = p.prev[mbase + i], nh = p.nhat[mbase + i];
        const cpx<T> fh = p.fhat ? p.fhat[mbase + i] : mk<T>(0, 0);
        const double st = stab_sym<STAB>(geo, p.udt, k2);
        const double iA = 1.0 / (p.ua0 + p.udt * k2 * (geo.a + k2 * k2) + st);
        const double f1 = -p.udt * xi * k2 * iA, f2 = (p.ua1 + st) * iA, f3 = p.ua2 * iA, f4 = p.udt * iA;
        const cpx<T> X = mk<T>(T(f1 * nh.x + f2 * cur.x + f3 * prv.x + f4 * fh.x),
                               T(f1 * nh.y + f2 * cur.y + f3 * prv.y + f4 * fh.y));
        p.out_new[mbase + i] = X;
        pair_partials<T, STAB>(X, cur, kx, k2, i == 0, geo, acc);
    }
    store_energy_partials<STAB>(acc, p.part + NPART_E * ((size_t)mem * gridDim.x + blockIdx.x));
}

// ------------------------------------------------------------------ forcing of a step

// f^{n+1} = sum_i c_i G_i on the half spectrum (the G_i transformed once); the scheme adds
// dt f^{n+1} to the right-hand side psi of the step (b2 = A^{-1} (psi + dt f)).
template <typename T>
__global__ void __launch_bounds__(256) k_force(ForceArgs<T> p) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < p.total;
         i += (long long)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k < p.terms; ++k) {
            const cpx<T> gk = p.g[(size_t)k * p.total + i];
            re += p.coef[k] * (double)gk.x;
            im += p.coef[k] * (double)gk.y;
        }
        p.out[i] = mk<T>(T(re), T(im));
    }
}

// ------------------------------------------------------------------ rows: real <-> half spectrum

// Two real rows per complex line: W = row0 + i row1, forward transform, split.
template <typename T, int NX, int EE, typename InT>
__global__ void __launch_bounds__(256) k_r2c_rows(RowArgs<T> p) {
    using PL = Plan<NX, EE>;
    constexpr int E = PL::E, P = PL::P;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw) + (threadIdx.x / P) * LdsLine<NX>::size;
    cpx<T>* ltw = reinterpret_cast<cpx<T>*>(smem_raw) + p.G * LdsLine<NX>::size;
    const int tid = threadIdx.x, g = tid / P, t = tid - g * P;
    const int row0 = (xcd_block(blockIdx.x, gridDim.x) * p.G + g) * 2;
    const bool act = row0 < p.nrows;
    const InT* in = reinterpret_cast<const InT*>(p.real[blockIdx.y]);
    cpx<T> v[1][E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int x = t + P * m;
        v[0][m] = act ? mk<T>(T(in[(size_t)row0 * NX + x]), T(in[(size_t)(row0 + 1) * NX + x])) : mk<T>(0, 0);
    }
    stage_twiddles<T, PL>(ltw, p.tw, p.tws);
    fft_run<T, PL, -1, 1>(v, lds, t, ltw);
    __syncthreads();
    line_store<T, PL, 1>(v, lds, t);
    __syncthreads();
    if (!act) return;
    cpx<T>* out = p.spec + (size_t)blockIdx.y * p.fs;
    const T half = T(0.5);
#pragma unroll
    for (int m = 0; m <= E / 2; ++m) {
        const int k = t + P * m;
        if (m == E / 2 && t != 0) break;
        const cpx<T> Vk = lds[lds_pad<NX>(k)];
        const cpx<T> Vm = lds[lds_pad<NX>((NX - k) & (NX - 1))];
        out[(size_t)k * p.nrows + row0] = mk<T>(half * (Vk.x + Vm.x), half * (Vk.y - Vm.y));
        out[(size_t)k * p.nrows + row0 + 1] = mk<T>(half * (Vk.y + Vm.y), half * (Vm.x - Vk.x));
    }
}

// Two half-spectrum rows -> one complex line -> inverse transform -> two real rows, scaled.
template <typename T, int NX, int EE, typename OutT>
__global__ void __launch_bounds__(256) k_c2r_rows(RowArgs<T> p) {
    using PL = Plan<NX, EE>;
    constexpr int E = PL::E, P = PL::P;
    constexpr int NXH = NX / 2 + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw) + (threadIdx.x / P) * LdsLine<NX>::size;
    cpx<T>* ltw = reinterpret_cast<cpx<T>*>(smem_raw) + p.G * LdsLine<NX>::size;
    const int tid = threadIdx.x, g = tid / P, t = tid - g * P;
    const int row0 = (xcd_block(blockIdx.x, gridDim.x) * p.G + g) * 2;
    const bool act = row0 < p.nrows;
    const cpx<T>* in = p.spec + (size_t)blockIdx.y * p.fs;
    const cpx<T>* h1 = in + (size_t)(act ? row0 : 0) * NXH;
    const cpx<T>* h2 = in + (size_t)(act ? row0 + 1 : 0) * NXH;
    cpx<T> v[1][E];
#pragma unroll
    for (int m = 0; m < E; ++m) v[0][m] = act ? load_packed<T, NX, false>(h1, h2, t + P * m, 0.0) : mk<T>(0, 0);
    stage_twiddles<T, PL>(ltw, p.tw, p.tws);
    fft_run<T, PL, +1, 1>(v, lds, t, ltw);
    if (!act) return;
    OutT* out = reinterpret_cast<OutT*>(p.real[blockIdx.y]);
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int x = t + P * m;
        out[(size_t)row0 * NX + x] = OutT((double)v[0][m].x * p.scale);
        out[(size_t)(row0 + 1) * NX + x] = OutT((double)v[0][m].y * p.scale);
    }
}

}  // namespace spfc
