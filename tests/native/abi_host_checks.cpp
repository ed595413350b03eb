// Host-only checks of the ABI code and the line-FFT schedule, built with the host
// AddressSanitizer and UndefinedBehaviorSanitizer (device code is not instrumented and no
// device is touched): every entry point that validates its arguments before any device
// work is called with good and bad arguments, the workspace sizes of every supported
// grid are computed, and the FFT schedule runs against a direct DFT.  Exit status 0 =
// all checks passed (a sanitizer report aborts with a non-zero status).
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "spfc.h"
#include "spfc_fno.h"

extern "C" int emu_fft_lines(int fp32, int n, int e, int dir, int c, const double* in, double* out);

static int failures = 0;
#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                               \
        }                                                             \
    } while (0)

static spfc_grid grid(int dim, int nx, int ny, int nz) {
    spfc_grid g{};
    g.dim = dim;
    g.n[0] = nx;
    g.n[1] = ny;
    g.n[2] = nz;
    g.L[0] = g.L[1] = g.L[2] = 10.0;
    return g;
}

static spfc_params params(int prec) {
    spfc_params p{};
    p.epsilon = 0.25;
    p.c4 = 1.0;
    p.startup = SPFC_STARTUP_SAV1;
    p.precision = prec;
    p.history = 16;
    p.energy_tol = 0.0;
    p.stab = 0.0;
    return p;
}

int main() {
    // workspace sizes: every supported 2-D grid, 3-D up to 512, both precisions
    for (int prec : {SPFC_FP64, SPFC_FP32}) {
        const spfc_params p = params(prec);
        for (int nx = 8; nx <= 1024; nx *= 2)
            for (int ny = 8; ny <= 1024; ny *= 4) {
                spfc_grid g = grid(2, nx, ny, 1);
                size_t b = 0;
                CHECK(spfc_workspace_bytes(&g, &p, &b) == SPFC_OK && b > 0);
            }
        for (int n = 8; n <= 512; n *= 2) {
            spfc_grid g = grid(3, n, n, n);
            size_t b = 0;
            CHECK(spfc_workspace_bytes(&g, &p, &b) == SPFC_OK && b > 0);
        }
    }
    // bad grids and parameters
    {
        spfc_params p = params(SPFC_FP64);
        size_t b = 0;
        for (int n : {0, 4, 12, 2048, -8}) {
            spfc_grid g = grid(2, n, 16, 1);
            CHECK(spfc_workspace_bytes(&g, &p, &b) == SPFC_E_INVAL);
        }
        spfc_grid g = grid(4, 16, 16, 16);
        CHECK(spfc_workspace_bytes(&g, &p, &b) == SPFC_E_INVAL);
        g = grid(2, 16, 16, 1);
        g.L[1] = -1.0;
        CHECK(spfc_workspace_bytes(&g, &p, &b) == SPFC_E_INVAL);
        g = grid(2, 16, 16, 1);
        p.epsilon = 1.0;
        CHECK(spfc_workspace_bytes(&g, &p, &b) == SPFC_E_INVAL);
        p = params(SPFC_FP64);
        p.c4 = NAN;
        CHECK(spfc_workspace_bytes(&g, &p, &b) == SPFC_E_INVAL);
        p = params(SPFC_FP64);
        p.stab = -1.0;
        CHECK(spfc_workspace_bytes(&g, &p, &b) == SPFC_E_INVAL);
        p = params(7);
        CHECK(spfc_workspace_bytes(&g, &p, &b) == SPFC_E_INVAL);
        CHECK(spfc_workspace_bytes(&g, nullptr, &b) == SPFC_E_INVAL);
        CHECK(spfc_workspace_bytes(nullptr, &p, &b) == SPFC_E_INVAL);
        p = params(SPFC_FP64);
        CHECK(spfc_workspace_bytes(&g, &p, nullptr) == SPFC_E_INVAL);
    }
    // batches: mixed sizes, then a member that disagrees on the start-up
    {
        std::vector<spfc_grid> gs = {grid(2, 128, 128, 1), grid(2, 256, 256, 1), grid(2, 128, 128, 1),
                                     grid(3, 16, 16, 16)};
        std::vector<spfc_params> ps(gs.size(), params(SPFC_FP64));
        ps[1].precision = SPFC_FP32;
        size_t b = 0;
        CHECK(spfc_batch_workspace_bytes((int)gs.size(), gs.data(), ps.data(), &b) == SPFC_OK && b > 0);
        ps[2].startup = SPFC_STARTUP_COPY;
        CHECK(spfc_batch_workspace_bytes((int)gs.size(), gs.data(), ps.data(), &b) == SPFC_E_INVAL);
        CHECK(spfc_batch_workspace_bytes(0, gs.data(), ps.data(), &b) == SPFC_E_INVAL);
    }
    // null contexts and pointers (checked before any device work)
    {
        double d = 0.0;
        int64_t i = 0;
        uint32_t f = 0;
        size_t s = 0;
        spfc_energy_t e{};
        spfc_record r{};
        CHECK(spfc_step(nullptr, 0.01, 1) == SPFC_E_INVAL);
        CHECK(spfc_step_forced(nullptr, 0.01, 1, nullptr) == SPFC_E_INVAL);
        CHECK(spfc_forcing_bytes(nullptr, 1, &s) == SPFC_E_INVAL);
        CHECK(spfc_set_forcing(nullptr, 0, nullptr, nullptr, 0) == SPFC_E_INVAL);
        CHECK(spfc_mass(nullptr, &d) == SPFC_E_INVAL);
        CHECK(spfc_energy(nullptr, &e) == SPFC_E_INVAL);
        CHECK(spfc_history(nullptr, 0, 1, &r) == SPFC_E_INVAL);
        CHECK(spfc_step_count(nullptr, &i) == SPFC_E_INVAL);
        CHECK(spfc_status(nullptr, &f) == SPFC_E_INVAL);
        CHECK(spfc_state_bytes(nullptr, &s) == SPFC_E_INVAL);
        CHECK(spfc_destroy(nullptr) == SPFC_E_INVAL);
        CHECK(spfc_batch_reset(nullptr, nullptr, nullptr) == SPFC_E_INVAL);
        CHECK(spfc_batch_get_phi_all(nullptr, nullptr, SPFC_FP64) == SPFC_E_INVAL);
        CHECK(spfc_batch_energies(nullptr, &e) == SPFC_E_INVAL);
        spfc_grid g = grid(2, 16, 16, 1);
        spfc_params p = params(SPFC_FP64);
        spfc_ctx* ctx = nullptr;
        CHECK(spfc_init(&g, &p, nullptr, nullptr, 0, nullptr, &ctx) == SPFC_E_INVAL && ctx == nullptr);
        for (int st = -1; st <= 6; ++st) CHECK(spfc_strerror(st) != nullptr);
    }
    // the surrogate's sizes and validation
    {
        int64_t count = 0;
        CHECK(spfc_fno_param_count(&count) == 0 && count == 4200801);
        for (int n : {64, 128, 256})
            for (int mb : {1, 32, 128})
                for (int tr : {0, 1}) {
                    spfc_fno_shape sh{n, mb, tr};
                    size_t b = 0;
                    CHECK(spfc_fno_workspace_bytes(&sh, &b) == 0 && b > 0);
                }
        for (spfc_fno_shape sh : {spfc_fno_shape{32, 4, 0}, spfc_fno_shape{64, 0, 0}, spfc_fno_shape{64, 129, 0},
                                  spfc_fno_shape{64, 4, 2}}) {
            size_t b = 0;
            CHECK(spfc_fno_workspace_bytes(&sh, &b) != 0);
        }
        CHECK(spfc_fno_destroy(nullptr) != 0);
    }
    // the line-FFT schedule against a direct DFT
    for (int fp32 : {0, 1})
        for (int n = 8; n <= 1024; n *= 2)
            for (int e : {4, 8, 16})
                for (int c : {1, 3}) {
                    std::vector<double> in(2 * c * n), out(2 * c * n);
                    for (size_t k = 0; k < in.size(); ++k) in[k] = std::sin(0.37 * k + 0.1 * n) + 0.25 * std::cos(1.3 * k);
                    CHECK(emu_fft_lines(fp32, n, e, -1, c, in.data(), out.data()) == 0);
                    double err = 0.0, mag = 0.0;
                    for (int l = 0; l < c; ++l)
                        for (int k = 0; k < n; k += (n > 64 ? 7 : 1)) {
                            std::complex<double> s = 0.0;
                            for (int j = 0; j < n; ++j) {
                                const double a = -2.0 * M_PI * (double)((long long)k * j % n) / n;
                                s += std::complex<double>(in[2 * (l * n + j)], in[2 * (l * n + j) + 1]) *
                                     std::complex<double>(std::cos(a), std::sin(a));
                            }
                            const std::complex<double> got(out[2 * (l * n + k)], out[2 * (l * n + k) + 1]);
                            err = std::fmax(err, std::abs(got - s));
                            mag = std::fmax(mag, std::abs(s));
                        }
                    // rounding grows like eps log2(n) (inputs rounded to the storage precision first)
                    const double tol = (fp32 ? 1.2e-7 : 2e-15) * std::log2((double)n) * mag;
                    if (!(err <= tol))
                        std::fprintf(stderr, "fft n=%d e=%d c=%d fp32=%d rel err %.3e\n", n, e, c, fp32, err / mag);
                    CHECK(err <= tol);
                }
    std::printf("host checks: %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
