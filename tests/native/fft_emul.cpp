// Host-side run of the line-FFT schedule of fft_core.hpp, thread by thread, for
// the CPU tests: the same pass code the kernels use, with the workgroup barriers
// replaced by running every thread's step before the next step starts.
#include <cstring>
#include <vector>
#include <cmath>
#include <array>

#include "../../paper_2012_15133_amd/csrc/fft_core.hpp"

using namespace spfc;

template <typename T, int N, int DIR, int C, int PASS>
static void emu_passes(std::vector<std::array<std::array<cpx<T>, Plan<N>::E>, C>>& regs, cpx<T>* lds,
                       const cpx<T>* tw, int tws) {
    constexpr int P = Plan<N>::P;
    using Reg = cpx<T>[C][Plan<N>::E];
    if constexpr (PASS > 0) {
        for (int t = 0; t < P; ++t) pass_store<T, N, C, PASS - 1>(*reinterpret_cast<Reg*>(&regs[t]), lds, t);
        for (int t = 0; t < P; ++t) pass_load<T, N, C, PASS>(*reinterpret_cast<Reg*>(&regs[t]), lds, t);
    }
    for (int t = 0; t < P; ++t) pass_compute<T, N, DIR, C, PASS>(*reinterpret_cast<Reg*>(&regs[t]), t, tw, tws);
    if constexpr (PASS + 1 < Plan<N>::NP) emu_passes<T, N, DIR, C, PASS + 1>(regs, lds, tw, tws);
}

template <typename T, int N, int DIR, int C>
static void emu(const double* in, double* out) {
    constexpr int E = Plan<N>::E, P = Plan<N>::P;
    std::vector<cpx<T>> tw(N);
    for (int j = 0; j < N; ++j) {
        long double a = -2.0L * 3.14159265358979323846264338327950288L * j / N;
        tw[j] = mk<T>(T(std::cos(a)), T(std::sin(a)));
    }
    std::vector<std::array<std::array<cpx<T>, E>, C>> regs(P);
    for (int t = 0; t < P; ++t)
        for (int c = 0; c < C; ++c)
            for (int m = 0; m < E; ++m) {
                const int e = t + P * m;
                regs[t][c][m] = mk<T>(T(in[2 * (c * N + e)]), T(in[2 * (c * N + e) + 1]));
            }
    std::vector<cpx<T>> lds(C * LdsLine<N>::size);
    emu_passes<T, N, DIR, C, 0>(regs, lds.data(), tw.data(), 1);
    for (int t = 0; t < P; ++t)
        for (int c = 0; c < C; ++c)
            for (int m = 0; m < E; ++m) {
                const int e = t + P * m;
                out[2 * (c * N + e)] = double(regs[t][c][m].x);
                out[2 * (c * N + e) + 1] = double(regs[t][c][m].y);
            }
}

template <typename T, int DIR, int C>
static int dispatch_n(int n, const double* in, double* out) {
    switch (n) {
        case 8: emu<T, 8, DIR, C>(in, out); return 0;
        case 16: emu<T, 16, DIR, C>(in, out); return 0;
        case 32: emu<T, 32, DIR, C>(in, out); return 0;
        case 64: emu<T, 64, DIR, C>(in, out); return 0;
        case 128: emu<T, 128, DIR, C>(in, out); return 0;
        case 256: emu<T, 256, DIR, C>(in, out); return 0;
        case 512: emu<T, 512, DIR, C>(in, out); return 0;
        case 1024: emu<T, 1024, DIR, C>(in, out); return 0;
        default: return 1;
    }
}

// in/out: C lines of n complex values (interleaved re, im), line-major.
extern "C" int emu_fft_lines(int fp32, int n, int dir, int c, const double* in, double* out) {
    if (c != 1 && c != 3) return 2;
    if (fp32) {
        if (dir < 0) return c == 1 ? dispatch_n<float, -1, 1>(n, in, out) : dispatch_n<float, -1, 3>(n, in, out);
        return c == 1 ? dispatch_n<float, 1, 1>(n, in, out) : dispatch_n<float, 1, 3>(n, in, out);
    }
    if (dir < 0) return c == 1 ? dispatch_n<double, -1, 1>(n, in, out) : dispatch_n<double, -1, 3>(n, in, out);
    return c == 1 ? dispatch_n<double, 1, 1>(n, in, out) : dispatch_n<double, 1, 3>(n, in, out);
}
