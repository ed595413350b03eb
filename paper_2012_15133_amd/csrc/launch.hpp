// Host-side launchers: pick the template instance for a line length and the
// workgroup shape (line groups per workgroup) for the kernels of kernels.hpp.
#pragma once

#include <algorithm>

#include "common.hpp"

namespace spfc {

// Shape of one launch of a line kernel.
struct LaunchShape {
    int E;          // values per thread (radix of the full passes)
    int G;          // line groups per workgroup
    int block;      // threads per workgroup
    int grid;       // workgroups per member
    size_t shmem;   // dynamic LDS bytes
    int members;    // batch members (grid y)
};

// Entries of the two staged twiddle tables of a line of length n (TwSplit<n>::size).
constexpr int tw_split_size(int n) { return (1 << (ilog2(n) / 2)) + n / (1 << (ilog2(n) / 2)); }
static_assert(tw_split_size(8) == TwSplit<8>::size && tw_split_size(256) == TwSplit<256>::size &&
                  tw_split_size(512) == TwSplit<512>::size && tw_split_size(1024) == TwSplit<1024>::size,
              "host LDS size of the twiddle tables");

// E values per thread (clamped to the line length), P = N / E threads per group,
// C complex lines per group, ngroups groups in total.  LDS: the groups' line
// buffers plus the two twiddle tables (about 2 sqrt(N) entries).
inline LaunchShape line_shape(int N, int C, size_t elem, int ngroups, int E = 16, int want_threads = 256,
                              size_t lds_cap = 65536) {
    E = std::min(E, N);
    if (N < 16) E = N;
    const int P = N / E;
    const size_t per = (size_t)C * (size_t)(N + N / 16) * elem;
    const size_t twb = (size_t)tw_split_size(N) * elem;
    int G = std::max(1, want_threads / P);
    while (G > 1 && (size_t)G * per + twb > lds_cap) --G;
    G = std::max(1, std::min(G, ngroups));
    LaunchShape s;
    s.E = E;
    s.G = G;
    s.block = G * P;
    s.grid = (ngroups + G - 1) / G;
    s.shmem = (size_t)G * per + twb;
    s.members = 1;
    return s;
}

template <typename T>
struct Kern {
    // stab: the stabilized-scheme variant (any member with a nonzero stabilization)
    // fin: the variant that closes the pending step inside the kernel (a.fin set)
    static hipError_t spec_inv(int nl, int dim, bool stab, bool fin, const SpecInvArgs<T>& a, const LaunchShape& s,
                               hipStream_t st);
    static hipError_t real_pass(int nx, int dim, bool fwd, bool beta, const RealArgs<T>& a, const LaunchShape& s,
                                hipStream_t st);
    // fold: also sum the real-space pass's E_1 partials into the forward partials (NPART_PF)
    static hipError_t spec_fwd(int nl, int dim, int mode, bool stab, bool fold, const SpecFwdArgs<T>& a,
                               const LaunchShape& s, hipStream_t st);
    static hipError_t pass(int nl, int dir, int omode, int c, const PassArgs<T>& a, const LaunchShape& s,
                           hipStream_t st);
    // the 3-D y passes of a step (k_ypass): dir +1 inverse (2 fields in, 3 out), -1 forward (3 in, 2 out)
    static hipError_t ypass(int nl, int dir, const PassArgs<T>& a, const LaunchShape& s, hipStream_t st);
    static hipError_t update(int dim, bool stab, const UpdateArgs<T>& a, int grid, int members, int block,
                             hipStream_t st);
    static hipError_t r2c_rows(int nx, const RowArgs<T>& a, const LaunchShape& s, hipStream_t st);
    static hipError_t force(const ForceArgs<T>& a, hipStream_t st);
    // values per thread available for line length n
    static bool has_E(int n, int E) { return n < 16 ? E == n : (E == 4 || E == 8 || E == 16); }
    static hipError_t c2r_rows(int nx, bool out_fp32, const RowArgs<T>& a, const LaunchShape& s, hipStream_t st);
};

hipError_t launch_finalize(const FinalizeArgs& a, int members, hipStream_t st);

}  // namespace spfc
