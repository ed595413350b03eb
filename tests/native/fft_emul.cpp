// Host-side run of the line-FFT schedule of fft_core.hpp, thread by thread, for
// the CPU tests: the same pass code the kernels use, with the workgroup barriers
// replaced by running every thread's step before the next step starts.
#include <cstring>
#include <vector>
#include <cmath>
#include <array>

#include "../../paper_2012_15133_amd/csrc/fft_core.hpp"

using namespace spfc;

template <typename T, typename PL, int DIR, int C, int PASS>
static void emu_passes(std::vector<std::array<std::array<cpx<T>, PL::E>, C>>& regs, cpx<T>* lds,
                       const cpx<T>* ptw) {
    constexpr int P = PL::P;
    using Reg = cpx<T>[C][PL::E];
    if constexpr (PASS > 0) {
        for (int t = 0; t < P; ++t) pass_store<T, PL, C, PASS - 1>(*reinterpret_cast<Reg*>(&regs[t]), lds, t);
        for (int t = 0; t < P; ++t) pass_load<T, PL, C, PASS>(*reinterpret_cast<Reg*>(&regs[t]), lds, t);
    }
    for (int t = 0; t < P; ++t) pass_compute<T, PL, DIR, C, PASS>(*reinterpret_cast<Reg*>(&regs[t]), t, ptw);
    if constexpr (PASS + 1 < PL::NP) emu_passes<T, PL, DIR, C, PASS + 1>(regs, lds, ptw);
}

template <typename T, int N, int EE, int DIR, int C>
static void emu(const double* in, double* out) {
    using PL = Plan<N, EE>;
    constexpr int E = PL::E, P = PL::P;
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
    std::vector<cpx<T>> ptw(N);
    build_twiddles<T, PL>(ptw.data(), tw.data(), 1, 0, 1);
    emu_passes<T, PL, DIR, C, 0>(regs, lds.data(), ptw.data());
    for (int t = 0; t < P; ++t)
        for (int c = 0; c < C; ++c)
            for (int m = 0; m < E; ++m) {
                const int e = t + P * m;
                out[2 * (c * N + e)] = double(regs[t][c][m].x);
                out[2 * (c * N + e) + 1] = double(regs[t][c][m].y);
            }
}

template <typename T, int EE, int DIR, int C>
static int dispatch_n(int n, const double* in, double* out) {
    switch (n) {
        case 8: emu<T, 8, 8, DIR, C>(in, out); return 0;
        case 16: emu<T, 16, EE, DIR, C>(in, out); return 0;
        case 32: emu<T, 32, EE, DIR, C>(in, out); return 0;
        case 64: emu<T, 64, EE, DIR, C>(in, out); return 0;
        case 128: emu<T, 128, EE, DIR, C>(in, out); return 0;
        case 256: emu<T, 256, EE, DIR, C>(in, out); return 0;
        case 512: emu<T, 512, EE, DIR, C>(in, out); return 0;
        case 1024: emu<T, 1024, EE, DIR, C>(in, out); return 0;
        default: return 1;
    }
}

template <typename T, int EE>
static int dispatch_dc(int n, int dir, int c, const double* in, double* out) {
    if (dir < 0) return c == 1 ? dispatch_n<T, EE, -1, 1>(n, in, out) : dispatch_n<T, EE, -1, 3>(n, in, out);
    return c == 1 ? dispatch_n<T, EE, 1, 1>(n, in, out) : dispatch_n<T, EE, 1, 3>(n, in, out);
}

// in/out: C lines of n complex values (interleaved re, im), line-major; e = values per thread.
extern "C" int emu_fft_lines(int fp32, int n, int e, int dir, int c, const double* in, double* out) {
    if (c != 1 && c != 3) return 2;
    if (e != 4 && e != 8 && e != 16) return 3;
    if (fp32) {
        if (e == 16) return dispatch_dc<float, 16>(n, dir, c, in, out);
        if (e == 8) return dispatch_dc<float, 8>(n, dir, c, in, out);
        return dispatch_dc<float, 4>(n, dir, c, in, out);
    }
    if (e == 16) return dispatch_dc<double, 16>(n, dir, c, in, out);
    if (e == 8) return dispatch_dc<double, 8>(n, dir, c, in, out);
    return dispatch_dc<double, 4>(n, dir, c, in, out);
}
