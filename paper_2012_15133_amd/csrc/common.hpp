// Types shared by the host driver and the kernels.
#pragma once

#include <cstdint>

#include "fft_core.hpp"

namespace spfc {

// Grid geometry and model constants in the form the kernels use.
struct Geo {
    int dim;
    int nx, ny, nz;       // points per axis (nz = 1 in 2-D)
    int nxh;              // nx/2 + 1: kept x wavenumbers of the half spectrum
    double k0x, k0y, k0z; // 2 pi / L_j
    double a, c4;
    double inv_npts;      // 1 / (nx ny nz)
    double cell;          // h^d
    double volume;        // |Omega|
    double pscale;        // |Omega| / N_total^2: inner product from two spectra (Parseval)
    double e1_const;      // (1 + 1/c4) |Omega|
    double stab;          // A of the stabilized scheme (0: plain scheme)
    double beta;          // coefficient of the quartic term (beta/4) phi^4 (0: the SPFC energy)
};

// Device-resident scalars of the run.  Written by one lane only (vector stores),
// read by later launches.  Two copies: a step's finish reads one and writes the
// other, so that the workgroups that still read the old values in the same
// launch never see a half-written block.
struct DevScalars {
    double xi;            // xi of the latest solved step (used by the pending update)
    double r_n;           // r of the newest state of the pair
    double r_nm1;         // r of the older state of the pair
    double energy_prev;   // modified energy of the newest finalized record
    double E1, p1, p2, ppsi, S;   // latest step
    double q_E1;          // E_1 of the latest query / start-up pass
    double q_norm[5];     // latest ||L^1/2 X||^2, ||L^1/2 (2X - Y)||^2, ||X||^2, ||Delta X||^2,
                          // <X - Y, -Delta_N (X - Y)>
    double mean;          // mean of the newest state
    unsigned int flags;   // sticky SPFC_FLAG_* bits
    unsigned int pad0;
    long long last_record;
    long long step_x;     // index of the newest state X of the pair (the record a finish writes)
    double pad[2];
};

struct Record {
    double energy, mean, r, xi, E1, p1, S, reserved;
};

enum : unsigned int {
    FLAG_NONFINITE = 1u,
    FLAG_E1_BELOW_OMEGA = 2u,
    FLAG_P1_POSITIVE = 4u,
    FLAG_ENERGY_RISE = 8u,
};

// Partial sums per workgroup (FP64):
//   P (forward pass): p1, p2, p_psi                                   3 per workgroup
//                     When a separate kernel closes the step (k_finalize), a fourth: the
//                     sum of a fixed slice of the real-space pass's E_1 partials
//                     (workgroup w of W takes B[w nB / W, (w+1) nB / W))  4 per workgroup
//   E (forward pass): ||L^1/2 X||^2, ||L^1/2 (2X - Y)||^2, ||X||^2,
//                     ||Delta X||^2, Re X(0) (only the owner adds it),
//                     <X - Y, -Delta_N (X - Y)>                         6 per workgroup
//   B (real-space pass): E_1 density sum                              1 per workgroup
//   Q (update / query passes): the same five as E for the pair they form
// Lines of a 3-D y-pass group that go through the transform's exchanges (and the output
// tile) at a time.
constexpr int YPASS_CH = 1;
constexpr int NPART_P = 3, NPART_PF = 4, NPART_E = 6;

// What a launch needs to finish the previous step (the SAV scalar) itself.  All
// arrays are those of member 0; member m's part starts m * (count per member)
// further on (see member_finish).
struct FinishIn {
    const double* partP;
    const double* partE;
    int nPE;                 // workgroups per member of the forward pass that wrote P and E
    const double* partB;
    int nB;                  // workgroups per member of the real-space pass
    const DevScalars* sc_in;
    DevScalars* sc_out;
    Record* hist;
    long long hist_cap;      // records per member
    int check_rise;
    double energy_tol;
};

// A batch of M independent runs of one grid size ("members") shares every launch:
// member m is blockIdx.y (blockIdx.x for the one-workgroup kernels); its fields
// start m * fs elements after member 0's, and its geometry and model constants are
// geos[m].  A single run is a batch of one.

// ------------------------------------------------------------------ kernel arguments

// Spectral state -> (optional pending update) -> gradient spectra -> inverse
// transform along the contiguous (last) axis, written rotated [L][a][b].
template <typename T>
struct SpecInvArgs {
    const cpx<T>* cur;      // X of the pair (or phi^n before the update)
    const cpx<T>* prev;     // Y of the pair (or phi^{n-1} before the update)
    const cpx<T>* nhat;     // N of the previous step (update only)
    cpx<T>* out_new;        // where the updated state goes (update only)
    cpx<T>* out[3];         // phihat and i kappa1 phihat of the line's axis, transformed
    const cpx<T>* tw;
    int tws;
    int nlines, B;          // lines = A * B, b fastest
    int G;                  // lines per workgroup
    int update;             // apply the pending update
    double ua0, ua1, ua2, udt;   // weights and dt of the step that produced nhat
    int fin;                // update: 1 = finish that step here (reduce its partials), 0 = read xi
    FinishIn fi;            // fin = 1: partials and scalar blocks; fin = 0: fi.sc_in->xi
    double e1, e2;          // phihat = e1 X + e2 Y
    int want_grad;          // 0: only the pair partials (no transform, no output)
    double* part;           // no update: NPART_E partials of (X, Y) per workgroup
    size_t fs;              // member field stride (elements)
    const Geo* geos;
    const cpx<T>* fhat;     // update: forcing spectrum of the pending step (or null)
};

// Rows of the half spectrum along x -> C2R (two real rows per complex line) ->
// pointwise SPFC flux -> R2C, written rotated [X][rows].
template <typename T>
struct RealArgs {
    const cpx<T>* in[3];
    cpx<T>* out[3];
    const cpx<T>* tw;
    int tws;
    int nrows;              // rows (a, b) in the input, b fastest
    int G;                  // row groups per workgroup
    double* part;           // E_1 partial per workgroup
    size_t fs;
    const Geo* geos;
};

// Flux spectra along the last axis -> forward transform -> N, the two solves
// and the inner products; the last workgroup finishes the step.
template <typename T>
struct SpecFwdArgs {
    const cpx<T>* in[3];
    const cpx<T>* X;
    const cpx<T>* Y;
    cpx<T>* nhat;           // SOLVE: N out
    cpx<T>* ghost_out;      // GHOST: phi^{-1} out
    const cpx<T>* tw;
    int tws;
    int nlines, B, G;
    double a0, a1, a2, dt, e1, e2;
    double* partP;          // NPART_P per workgroup
    double* partE;          // NPART_E per workgroup
    const double* partB;    // FOLD: the real-space pass's E_1 partials (nB per member), folded
    int nB;                 // into partP (NPART_PF per workgroup)
    size_t fs;
    const Geo* geos;
    const cpx<T>* fhat;     // SOLVE_FORCED: forcing spectrum f^{n+1} of this step
};

// Generic batched line transform along the contiguous axis, with the output
// written in place ([a][b][L]), swapped ([a][L][b]) or rotated ([L][a][b]).
enum { OUT_KEEP = 0, OUT_SWAP = 1, OUT_ROTATE = 2 };

template <typename T>
struct PassArgs {
    const cpx<T>* in[3];
    cpx<T>* out[3];
    const cpx<T>* tw;
    int tws;
    int nlines, B, G;
    size_t fs;
    const Geo* geos;        // the 3-D y passes of a step (their y symbols); else unused
};

// Real rows <-> half-spectrum rows (set-up and queries), for up to ROW_TAB members in
// one launch: member y = blockIdx.y has its real field at real[y] (caller memory) and its
// half spectrum at spec + y * fs (workspace).
constexpr int ROW_TAB = 64;
template <typename T>
struct RowArgs {
    cpx<T>* spec;
    size_t fs;
    const cpx<T>* tw;
    int tws;
    int nrows, G;
    double scale;
    void* real[ROW_TAB];
};

// Pending update applied elementwise (end of a run of steps).
template <typename T>
struct UpdateArgs {
    const cpx<T>* cur;
    const cpx<T>* prev;
    const cpx<T>* nhat;
    cpx<T>* out_new;
    long long total;         // complex entries of one spectrum
    int NL, B;               // line length (last axis) and b extent
    double ua0, ua1, ua2, udt;
    int fin;
    FinishIn fi;
    double* part;            // NPART_E per workgroup
    size_t fs;
    const Geo* geos;
    const cpx<T>* fhat;      // forcing spectrum of the pending step (or null)
};

// Forcing spectrum of one step: out = sum_i coef[i] g[i] (terms spectra of one member).
template <typename T>
struct ForceArgs {
    cpx<T>* out;
    const cpx<T>* g;
    int terms;
    const double* coef;      // device, `terms` values
    long long total;         // complex entries of one spectrum
};

enum { FWD_SOLVE = 0, FWD_GHOST = 1, FWD_SOLVE_FORCED = 2 };

enum { FIN_STATE = 0, FIN_QUERY = 1, FIN_GHOST_R0 = 2, FIN_GHOST_RM1 = 3, FIN_RESTART = 4, FIN_STEP = 5 };

// One workgroup per member (blockIdx.x = member).
struct FinalizeArgs {
    int mode;
    const double* partQ;    // NPART_E per workgroup (state / query modes)
    int nQ;                 // workgroups per member that wrote Q
    const double* partB;
    int nB;
    double a0, a1, a2, dt;  // FIN_STEP: weights and dt of the step; FIN_STATE: dt of the last step
    FinishIn fi;            // FIN_STEP
    DevScalars* sc;         // other modes: updated in place
    Record* hist;
    long long hist_cap;
    int check_rise;
    double energy_tol;
    const Geo* geos;
};

}  // namespace spfc
