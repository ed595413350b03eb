// Host driver and C ABI (include/spfc.h): validation, workspace carving, the
// per-step launch sequence, start-up, queries, checkpoints, graph replay of the
// steady steps, and batches of independent runs ("members") of one grid size
// that share every launch.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "launch.hpp"
#include "trace.hpp"
#include "spfc.h"

using namespace spfc;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool pow2_ok(int n) { return n >= 8 && n <= 1024 && (n & (n - 1)) == 0; }

enum Role { R_SPEC_INV = 0, R_MID_INV, R_REAL, R_MID_FWD, R_SPEC_FWD, R_FINAL, R_COUNT };
const char* const kRoleNames[R_COUNT] = {"spec_inv", "pass_y_inv", "real_pass", "pass_y_fwd", "spec_fwd",
                                         "step_finalize"};

struct Sizes {
    int dim, nx, ny, nz, nxh;
    size_t elem;
    bool beta = false;   // the quartic term: the real-space pass carries the rows of phi
};

struct Shapes {
    LaunchShape A, B, Cf, midI, midF, r2c, keep, swapInit, rot, swapGet, c2r;
    int updGrid;
};

struct Layout {
    size_t F;            // bytes of one half-spectrum field of one member
    size_t fs;           // elements of one half-spectrum field of one member
    size_t field_bytes;  // bytes of one field region (all members)
    size_t sc_bytes;     // bytes of one copy of the scalar blocks (all members)
    size_t off_slot[2], off_nhat, off_bufA, off_bufB, off_tw, off_partP, off_partE, off_partB, off_partQ, off_geo,
        off_sc, off_hist;
    size_t total;
    int ntab;
};

// Launch plan of the step kernels: values per thread (E) and target threads per
// workgroup for each role.  Overridable with SPFC_PLAN="inv=E/T,real=E/T,fwd=E/T,mid=E/T"
// (and "finsep" to close every step in a separate kernel).  The 3-D inverse pass and y
// passes take workgroups of up to 512 threads (their built-in size), the other kernels up
// to 256.
constexpr int WIDE_T_MAX = 512, T_MAX = 256;
struct RolePlan {
    int E = 8, T = 256;
};
struct TunePlan {
    RolePlan inv, real, fwd, mid{8, WIDE_T_MAX};
    int fin_in_kernel = 1;  // allow closing each step inside the next update kernel
};

// largest workgroup of a role (0 inv, 1 real, 2 fwd, 3 mid) in `dim` dimensions
constexpr int role_t_max(int role, int dim) { return (role == 3 || (role == 0 && dim == 3)) ? WIDE_T_MAX : T_MAX; }

void parse_role(const char* spec, const char* key, RolePlan& r, int tmax) {
    const char* p = std::strstr(spec, key);
    if (!p) return;
    p += std::strlen(key);
    if (*p != '=') return;
    int e = 0, t = 0;
    if (std::sscanf(p + 1, "%d/%d", &e, &t) >= 1) {
        if (e == 4 || e == 8 || e == 16) r.E = e;
        if (t >= 64 && t <= tmax) r.T = t;
    }
}

TunePlan tune_plan(int dim) {
    TunePlan tp;
    if (dim == 3) tp.inv.T = WIDE_T_MAX;
    if (const char* env = std::getenv("SPFC_PLAN")) {
        parse_role(env, "inv", tp.inv, role_t_max(0, dim));
        parse_role(env, "real", tp.real, role_t_max(1, dim));
        parse_role(env, "fwd", tp.fwd, role_t_max(2, dim));
        parse_role(env, "mid", tp.mid, role_t_max(3, dim));
        if (std::strstr(env, "finsep")) tp.fin_in_kernel = 0;
    }
    return tp;
}

Sizes sizes_of(const spfc_grid& g, int prec) {
    Sizes s;
    s.dim = g.dim;
    s.nx = g.n[0];
    s.ny = g.n[1];
    s.nz = g.dim == 3 ? g.n[2] : 1;
    s.nxh = s.nx / 2 + 1;
    s.elem = prec == SPFC_FP32 ? 2 * sizeof(float) : 2 * sizeof(double);
    return s;
}

Shapes shapes_of(const Sizes& s, int M, const TunePlan& tp) {
    Shapes h{};
    const int d = s.dim;
    const int nl = d == 2 ? s.ny : s.nz;               // contiguous spectral axis
    const int nlines = d == 2 ? s.nxh : s.nxh * s.ny;  // spectral lines per member
    // the spectral passes carry two lines each (phihat and one derivative; two flux fields)
    h.A = line_shape(nl, d == 3 ? 1 : 2, s.elem, nlines, tp.inv.E, tp.inv.T);   // 3-D: one line buffer per group
    h.Cf = line_shape(nl, 2, s.elem, nlines, tp.fwd.E, tp.fwd.T);
    // real-space pass: lines per row group (2-D one row per group; 3-D and with the
    // quartic term two rows, plus the line of phi)
    const int rowgroups = (d == 2 && !s.beta) ? s.ny : s.nz * s.ny / 2;
    const int cB = (d == 2 ? 1 : 3) + (s.beta ? (d == 2 ? 2 : 1) : 0);
    h.B = line_shape(s.nx, cB, s.elem, rowgroups, tp.real.E, tp.real.T);
    if (d == 3) {
        h.midI = line_shape(s.ny, YPASS_CH, s.elem, s.nz * s.nxh, tp.mid.E, tp.mid.T);
        h.midF = line_shape(s.ny, YPASS_CH, s.elem, s.nxh * s.nz, tp.mid.E, tp.mid.T);
        h.swapInit = line_shape(s.ny, 1, s.elem, s.nxh * s.nz);
        h.swapGet = line_shape(s.ny, 1, s.elem, s.nz * s.nxh);
    }
    h.r2c = line_shape(s.nx, 1, s.elem, s.ny * s.nz / 2);
    h.c2r = line_shape(s.nx, 1, s.elem, s.ny * s.nz / 2);
    h.keep = line_shape(nl, 1, s.elem, nlines);
    h.rot = line_shape(nl, 1, s.elem, nlines);
    // the step kernels cover every member in one launch (grid y)
    for (LaunchShape* x : {&h.A, &h.Cf, &h.B, &h.midI, &h.midF}) x->members = M;
    const long long total = (long long)s.nxh * s.ny * s.nz;
    const long long cap = std::max(64, 2048 / M);
    h.updGrid = (int)std::max<long long>(1, std::min<long long>((total + 255) / 256, cap));
    return h;
}

// Partial-sum buffers are sized for any launch plan (one line group per workgroup
// gives the most workgroups), so that a context can change its plan in place.
Layout layout_of(const Sizes& s0, int64_t hist_cap, int M) {
    TunePlan widest;
    widest.inv.T = widest.real.T = widest.fwd.T = widest.mid.T = 1;
    Sizes s = s0;
    s.beta = false;   // one real-space row per workgroup in 2-D: the most partials of either variant
    const Shapes h = shapes_of(s, M, widest);
    Layout L{};
    L.fs = (size_t)s.nxh * s.ny * s.nz;
    L.F = L.fs * s.elem;
    L.field_bytes = align_up(L.F * M);
    size_t o = 0;
    L.off_slot[0] = o; o += L.field_bytes;
    L.off_slot[1] = o; o += L.field_bytes;
    L.off_nhat = o; o += L.field_bytes;
    L.off_bufA = o; o += 3 * L.field_bytes;
    L.off_bufB = o; o += 3 * L.field_bytes;
    L.ntab = std::max(s.nx, std::max(s.ny, s.nz));
    L.off_tw = o; o += align_up((size_t)L.ntab * s.elem);
    const int nQ = std::max(h.A.grid, h.updGrid);
    L.off_partP = o; o += align_up((size_t)M * h.Cf.grid * NPART_PF * sizeof(double));
    L.off_partE = o; o += align_up((size_t)M * h.Cf.grid * NPART_E * sizeof(double));
    L.off_partB = o; o += align_up((size_t)M * h.B.grid * sizeof(double));
    L.off_partQ = o; o += align_up((size_t)M * nQ * NPART_E * sizeof(double));
    L.off_geo = o; o += align_up((size_t)M * sizeof(Geo));
    L.sc_bytes = align_up((size_t)M * sizeof(DevScalars));
    L.off_sc = o; o += 2 * L.sc_bytes;
    L.off_hist = o; o += align_up((size_t)M * hist_cap * sizeof(Record));
    L.total = o;
    return L;
}

int validate(const spfc_grid* g, const spfc_params* p) {
    if (!g || !p) return SPFC_E_INVAL;
    if (g->dim != 2 && g->dim != 3) return SPFC_E_INVAL;
    for (int j = 0; j < g->dim; ++j) {
        if (!pow2_ok(g->n[j])) return SPFC_E_INVAL;
        if (!(g->L[j] > 0.0) || !std::isfinite(g->L[j])) return SPFC_E_INVAL;
    }
    if (!std::isfinite(p->epsilon) || !(1.0 - p->epsilon > 0.0)) return SPFC_E_INVAL;
    if (!std::isfinite(p->c4) || !(p->c4 > 0.0)) return SPFC_E_INVAL;
    if (p->startup < SPFC_STARTUP_SAV1 || p->startup > SPFC_STARTUP_COPY) return SPFC_E_INVAL;
    if (p->precision != SPFC_FP64 && p->precision != SPFC_FP32) return SPFC_E_INVAL;
    if (p->history < 1) return SPFC_E_INVAL;
    if (!std::isfinite(p->energy_tol)) return SPFC_E_INVAL;
    if (!std::isfinite(p->stab) || p->stab < 0.0) return SPFC_E_INVAL;
    if (!std::isfinite(p->beta) || p->beta < 0.0) return SPFC_E_INVAL;
    return SPFC_OK;
}

Geo make_geo(const spfc_grid& g, const spfc_params& prm) {
    Geo geo{};
    geo.dim = g.dim;
    geo.nx = g.n[0];
    geo.ny = g.n[1];
    geo.nz = g.dim == 3 ? g.n[2] : 1;
    geo.nxh = geo.nx / 2 + 1;
    const double twopi = 6.283185307179586476925286766559;
    geo.k0x = twopi / g.L[0];
    geo.k0y = twopi / g.L[1];
    geo.k0z = g.dim == 3 ? twopi / g.L[2] : 0.0;
    geo.a = 1.0 - prm.epsilon;
    geo.c4 = prm.c4;
    const double npts = (double)geo.nx * geo.ny * geo.nz;
    geo.inv_npts = 1.0 / npts;
    const double vol = g.L[0] * g.L[1] * (g.dim == 3 ? g.L[2] : 1.0);
    geo.volume = vol;
    geo.cell = vol / npts;
    geo.pscale = vol / (npts * npts);
    geo.e1_const = (1.0 + 1.0 / prm.c4) * vol;
    geo.stab = prm.stab;
    geo.beta = prm.beta;
    return geo;
}

struct CkptHeader {
    uint64_t magic;
    int64_t step;
    double dt_prev;
    int32_t started, slot_same, prec, dim;
    int32_t n[3];
    int32_t pad;
    DevScalars sc;
};
constexpr uint64_t kMagic = 0x5350464353415633ull;

}  // namespace

// One grid size and precision; M members advance together (a single run is M = 1).
struct spfc_ctx {
    spfc_params prm;        // shared by the members: startup, precision, history, energy_tol
    int M;
    std::vector<Geo> geos;  // per member (host copy of the device array)
    Sizes sz;
    TunePlan plan;
    Shapes sh;
    Layout lay;
    hipStream_t stream;
    char* ws;
    int slotX, slotY;  // slots of the newest (X) and older (Y) state of the pair
    int64_t step;      // index of the newest state
    double dt_prev;
    bool started;
    bool broken;
    double energy_tol;
    int cur_sc;        // which of the two scalar-block copies holds the latest values
    bool stab;         // some member uses the stabilized scheme: launch the stabilized kernels
    bool fin_in;       // close each step inside the next update kernel
    // graph replay of two steady steps
    bool use_graph;
    char* force_buf = nullptr;   // caller memory: the combined forcing spectrum, then its terms
    int force_terms = 0;
    std::vector<std::pair<std::tuple<double, int, int, int>, hipGraphExec_t>> graphs;  // newest last
    int64_t graph_gen = 0;   // counts drop_graph calls: a batch graph records the values it was captured at
    // profiling
    bool profiling;
    std::vector<hipEvent_t> ev_pool;
    struct EvUse {
        int role, reps;
        hipEvent_t a, b;
    };
    std::vector<EvUse> ev_used;
    int reps;            // launches per timed kernel call (1; more in spfc_time_kernels)
    int64_t timed_from;  // first step of a call whose kernels are timed
    double role_ms[R_COUNT];
    int64_t role_n[R_COUNT];

    char* slot(int i) const { return ws + lay.off_slot[i]; }
    char* nhat() const { return ws + lay.off_nhat; }
    char* bufA(int j) const { return ws + lay.off_bufA + j * lay.field_bytes; }
    char* bufB(int j) const { return ws + lay.off_bufB + j * lay.field_bytes; }
    char* tw() const { return ws + lay.off_tw; }
    double* partP() const { return reinterpret_cast<double*>(ws + lay.off_partP); }
    double* partE() const { return reinterpret_cast<double*>(ws + lay.off_partE); }
    double* partB() const { return reinterpret_cast<double*>(ws + lay.off_partB); }
    double* partQ() const { return reinterpret_cast<double*>(ws + lay.off_partQ); }
    const Geo* dgeos() const { return reinterpret_cast<const Geo*>(ws + lay.off_geo); }
    DevScalars* scb(int i) const { return reinterpret_cast<DevScalars*>(ws + lay.off_sc + i * lay.sc_bytes); }
    DevScalars* sc(int m = 0) const { return scb(cur_sc) + m; }
    Record* hist(int m = 0) const { return reinterpret_cast<Record*>(ws + lay.off_hist) + (size_t)m * prm.history; }
    size_t moff(int m) const { return (size_t)m * lay.F; }
    int nl() const { return sz.dim == 2 ? sz.ny : sz.nz; }
    int nlines() const { return sz.dim == 2 ? sz.nxh : sz.nxh * sz.ny; }
    int lineB() const { return sz.dim == 2 ? sz.nxh : sz.ny; }
};

// A batch: one context per (grid size, precision) class of members.  With several
// classes each steps on a stream of its own (default priority), forked from the batch's
// stream at the start of spfc_batch_step and joined back at its end, so that the classes'
// kernels overlap on the device; every other call runs the classes on the batch's stream.
struct spfc_batch {
    std::vector<spfc_ctx*> cls;
    std::vector<std::pair<int, int>> where;  // member -> (class, index within the class)
    std::vector<std::vector<int>> members;   // class -> member indices
    std::vector<size_t> npts;                // member -> grid points
    hipStream_t stream = nullptr;            // the caller's stream
    std::vector<hipStream_t> cstream;        // one per class (several classes only)
    std::vector<hipEvent_t> join;            // one per class
    hipEvent_t fork = nullptr;
    // graph replay with several classes: one graph holds two steady steps of every class,
    // each class on a branch of its own; keyed by dt and every class's slot pair,
    // scalar-block parity and graph generation
    bool use_graph = false;
    std::vector<std::pair<std::vector<int64_t>, hipGraphExec_t>> graphs;  // newest last
};

namespace {

#define CK(x)                     \
    do {                          \
        hipError_t e_ = (x);      \
        if (e_ != hipSuccess) {   \
            ctx->broken = true;   \
            return SPFC_E_DEVICE; \
        }                         \
    } while (0)

// ---------------------------------------------------------------- profiling

hipEvent_t take_event(spfc_ctx* ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int drain_events(spfc_ctx* ctx) {
    if (ctx->ev_used.empty()) return SPFC_OK;
    CK(hipStreamSynchronize(ctx->stream));
    for (auto& u : ctx->ev_used) {
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, u.a, u.b));
        ctx->role_ms[u.role] += ms / u.reps;
        ctx->role_n[u.role] += 1;
        ctx->ev_pool.push_back(u.a);
        ctx->ev_pool.push_back(u.b);
    }
    ctx->ev_used.clear();
    return SPFC_OK;
}

// HIP events around the launches of one kernel role on the context stream.
// reps() launches go between the two events (more than one only inside
// spfc_time_kernels, which restores the run state afterwards).
struct Timed {
    spfc_ctx* ctx;
    int role;
    bool on;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(spfc_ctx* c, int r, bool timed) : ctx(c), role(r), on(timed && c->profiling) {
        if (on) {
            a = take_event(ctx);
            b = take_event(ctx);
            if (a && b) (void)hipEventRecord(a, ctx->stream);
        }
    }
    int reps() const { return on ? ctx->reps : 1; }
    ~Timed() {
        if (a && b) {
            (void)hipEventRecord(b, ctx->stream);
            ctx->ev_used.push_back({role, reps(), a, b});
        }
    }
};

void drop_graph(spfc_ctx* ctx) {
    for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
    ctx->graphs.clear();
    ++ctx->graph_gen;
}

void drop_batch_graphs(spfc_batch* b) {
    for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
    b->graphs.clear();
}

// Dynamic LDS of every launch shape of the plan within the device limit.
bool plan_fits(const Sizes& sz, int M, const TunePlan& tp, size_t lds_max) {
    const Shapes h = shapes_of(sz, M, tp);
    for (const LaunchShape* x : {&h.A, &h.B, &h.Cf, &h.midI, &h.midF, &h.r2c, &h.keep, &h.swapInit, &h.rot,
                                 &h.swapGet, &h.c2r})
        if (x->shmem > lds_max) return false;
    return true;
}

size_t device_lds_max() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 65536;
    return (size_t)v;
}

// Launch plan of a context: shapes of the step kernels and whether each step is
// closed inside the next update kernel.  That makes every workgroup of the update
// kernel read its member's partial sums: worth it while that re-read is small (the
// update-and-inverse kernel's workgroups each step; the elementwise update that ends a
// call re-reads them once per call).
void set_plan(spfc_ctx* ctx, const TunePlan& tp) {
    drop_graph(ctx);
    ctx->plan = tp;
    ctx->sh = shapes_of(ctx->sz, ctx->M, tp);
    const Shapes& h = ctx->sh;
    const double reread = (double)ctx->M * h.A.grid * (h.B.grid + NPART_P * h.Cf.grid) * 8.0;
    ctx->fin_in = tp.fin_in_kernel != 0 && reread <= 48.0e6;
}

// ---------------------------------------------------------------- pipeline (one precision)

// Weights of the steady BDF2 step (eq. scheme-SAV-1) and of the extrapolation 2X - Y.
constexpr double kA0 = 1.5, kA1 = 2.0, kA2 = -0.5, kE1 = 2.0, kE2 = -1.0;

// Pending step (weights, dt, rise check) whose scalar is still to be solved.
struct Pending {
    bool open = false;
    double a0 = 0, a1 = 0, a2 = 0, dt = 0;
    int check = 0;
    bool forced = false;   // its right-hand side holds dt f (spectrum in force_buf)
};

// State of one call of n steps of size dt on a context (Pipe::run_begin ... run_end).
struct StepRun {
    Pending pend;
    bool restart = false;
    bool first_order = false;
    int64_t i = 0;   // steps of this call issued so far
};

template <typename T>
struct Pipe {
    using C = cpx<T>;
    spfc_ctx* ctx;

    // What a launch needs to close the step whose N is pending (all members).
    FinishIn finish_in(int check_rise) {
        FinishIn f{};
        f.partP = ctx->partP();
        f.partE = ctx->partE();
        f.nPE = ctx->sh.Cf.grid;
        // the real-space partials are read by the close itself inside the next kernel, and
        // folded into the forward pass's partials when a separate kernel closes the step
        f.partB = ctx->partB();
        f.nB = ctx->fin_in ? ctx->sh.B.grid : 0;
        f.sc_in = ctx->scb(ctx->cur_sc);
        f.sc_out = ctx->scb(1 - ctx->cur_sc);
        f.hist = ctx->hist();
        f.hist_cap = ctx->prm.history;
        f.check_rise = check_rise;
        f.energy_tol = ctx->energy_tol;
        return f;
    }

    // spectral state (cur, prev) -> gradient transforms along the last axis -> bufA.
    // With `pend.open` the kernel first applies the pending update (closing that
    // step itself when ctx->fin_in).
    int spec_inv(const char* cur, const char* prev, char* out_new, const Pending& pend, double e1, double e2,
                 bool want_grad, bool timed) {
        SpecInvArgs<T> a{};
        a.cur = (const C*)cur;
        a.prev = (const C*)prev;
        a.nhat = (const C*)ctx->nhat();
        a.out_new = (C*)out_new;
        for (int j = 0; j < 3; ++j) a.out[j] = (C*)ctx->bufA(j);
        a.tw = (const C*)ctx->tw();
        a.tws = ctx->lay.ntab / ctx->nl();
        a.nlines = ctx->nlines();
        a.B = ctx->lineB();
        a.G = ctx->sh.A.G;
        a.update = pend.open ? 1 : 0;
        a.ua0 = pend.a0;
        a.ua1 = pend.a1;
        a.ua2 = pend.a2;
        a.udt = pend.dt;
        a.fin = (pend.open && ctx->fin_in) ? 1 : 0;
        a.fi = finish_in(pend.check);
        a.e1 = e1;
        a.e2 = e2;
        a.want_grad = want_grad ? 1 : 0;
        a.part = ctx->partQ();
        a.fs = ctx->lay.fs;
        a.geos = ctx->dgeos();
        a.fhat = (pend.open && pend.forced) ? (const C*)ctx->force_buf : nullptr;
        {
            Timed tm(ctx, R_SPEC_INV, timed);
            for (int r = 0; r < tm.reps(); ++r)
                CK(Kern<T>::spec_inv(ctx->nl(), ctx->sz.dim, ctx->stab, a.fin != 0, a, ctx->sh.A, ctx->stream));
        }
        if (a.fin) ctx->cur_sc = 1 - ctx->cur_sc;
        return SPFC_OK;
    }

    // 3-D middle pass along y: in -> out, [a][b][Y] -> [a][Y][b]; inverse 2 fields in, 3
    // out; forward 3 in, 2 out
    int mid(int dir, char* const* in, char* const* out, const LaunchShape& s, int nlines, int B, int role,
            bool timed) {
        PassArgs<T> a{};
        a.geos = ctx->dgeos();
        for (int j = 0; j < 3; ++j) {
            a.in[j] = (const C*)in[j];
            a.out[j] = (C*)out[j];
        }
        a.tw = (const C*)ctx->tw();
        a.tws = ctx->lay.ntab / ctx->sz.ny;
        a.nlines = nlines;
        a.B = B;
        a.G = s.G;
        a.fs = ctx->lay.fs;
        Timed tm(ctx, role, timed);
        for (int r = 0; r < tm.reps(); ++r) CK(Kern<T>::ypass(ctx->sz.ny, dir, a, s, ctx->stream));
        return SPFC_OK;
    }

    // gradient rows -> flux spectra (or E_1 only)
    int real_pass(char* const* in, char* const* out, bool fwd, bool timed) {
        RealArgs<T> a{};
        for (int j = 0; j < 3; ++j) {
            a.in[j] = (const C*)in[j];
            a.out[j] = (C*)out[j];
        }
        a.tw = (const C*)ctx->tw();
        a.tws = ctx->lay.ntab / ctx->sz.nx;
        a.nrows = ctx->sz.ny * ctx->sz.nz;
        a.G = ctx->sh.B.G;
        a.part = ctx->partB();
        a.fs = ctx->lay.fs;
        a.geos = ctx->dgeos();
        Timed tm(ctx, R_REAL, timed);
        for (int r = 0; r < tm.reps(); ++r)
            CK(Kern<T>::real_pass(ctx->sz.nx, ctx->sz.dim, fwd, ctx->sz.beta, a, ctx->sh.B, ctx->stream));
        return SPFC_OK;
    }

    int spec_fwd(char* const* in, const char* X, const char* Y, int mode, char* ghost_out, double a0, double a1,
                 double a2, double dt, double e1, double e2, bool timed, const char* fhat = nullptr) {
        SpecFwdArgs<T> a{};
        a.fhat = (const C*)fhat;
        for (int j = 0; j < 3; ++j) a.in[j] = (const C*)in[j];
        a.X = (const C*)X;
        a.Y = (const C*)Y;
        a.nhat = (C*)ctx->nhat();
        a.ghost_out = (C*)ghost_out;
        a.tw = (const C*)ctx->tw();
        a.tws = ctx->lay.ntab / ctx->nl();
        a.nlines = ctx->nlines();
        a.B = ctx->lineB();
        a.G = ctx->sh.Cf.G;
        a.a0 = a0;
        a.a1 = a1;
        a.a2 = a2;
        a.dt = dt;
        a.e1 = e1;
        a.e2 = e2;
        a.partP = ctx->partP();
        a.partE = ctx->partE();
        a.partB = ctx->partB();
        a.nB = ctx->fin_in ? 0 : ctx->sh.B.grid;
        a.fs = ctx->lay.fs;
        a.geos = ctx->dgeos();
        Timed tm(ctx, R_SPEC_FWD, timed);
        for (int r = 0; r < tm.reps(); ++r)
            CK(Kern<T>::spec_fwd(ctx->nl(), ctx->sz.dim, mode, ctx->stab, a.nB > 0, a, ctx->sh.Cf, ctx->stream));
        return SPFC_OK;
    }

    // one workgroup per member: close a step (FIN_STEP) or a state / query pass
    int finalize(int mode, int nQ, int check_rise, const Pending* pend = nullptr, bool timed = false,
                 double dt = 0.0) {
        FinalizeArgs f{};
        f.mode = mode;
        f.dt = dt;
        f.partQ = ctx->partQ();
        f.nQ = nQ;
        f.partB = ctx->partB();
        f.nB = ctx->sh.B.grid;
        if (pend) {
            f.a0 = pend->a0;
            f.a1 = pend->a1;
            f.a2 = pend->a2;
            f.dt = pend->dt;
            f.fi = finish_in(pend->check);
        }
        f.sc = ctx->sc();
        f.hist = ctx->hist();
        f.hist_cap = ctx->prm.history;
        f.check_rise = check_rise;
        f.energy_tol = ctx->energy_tol;
        f.geos = ctx->dgeos();
        {
            Timed tm(ctx, R_FINAL, timed);
            for (int r = 0; r < tm.reps(); ++r) CK(launch_finalize(f, ctx->M, ctx->stream));
        }
        if (mode == FIN_STEP) ctx->cur_sc = 1 - ctx->cur_sc;
        return SPFC_OK;
    }

    // E_1 of the state `field` (and the energy norms of (field, prev)) -> finalize(mode)
    int e1_pass(const char* field, const char* prev, int fin_mode) {
        int rc;
        if ((rc = spec_inv(field, prev, nullptr, Pending{}, 1.0, 0.0, true, false))) return rc;
        char* bA[3] = {ctx->bufA(0), ctx->bufA(1), ctx->bufA(2)};
        char* bB[3] = {ctx->bufB(0), ctx->bufB(1), ctx->bufB(2)};
        if (ctx->sz.dim == 3) {
            if ((rc = mid(+1, bA, bB, ctx->sh.midI, ctx->sz.nz * ctx->sz.nxh, ctx->sz.nxh, R_MID_INV, false)))
                return rc;
            if ((rc = real_pass(bB, bA, false, false))) return rc;
        } else {
            if ((rc = real_pass(bA, bB, false, false))) return rc;
        }
        return finalize(fin_mode, ctx->sh.A.grid, 0);
    }

    // gradient spectra in bufA -> flux spectra; returns where they are
    int flux(bool timed, char** out) {
        int rc;
        char* bA[3] = {ctx->bufA(0), ctx->bufA(1), ctx->bufA(2)};
        char* bB[3] = {ctx->bufB(0), ctx->bufB(1), ctx->bufB(2)};
        if (ctx->sz.dim == 3) {
            if ((rc = mid(+1, bA, bB, ctx->sh.midI, ctx->sz.nz * ctx->sz.nxh, ctx->sz.nxh, R_MID_INV, timed)))
                return rc;
            if ((rc = real_pass(bB, bA, true, timed))) return rc;
            if ((rc = mid(-1, bA, bB, ctx->sh.midF, ctx->sz.nxh * ctx->sz.nz, ctx->sz.nz, R_MID_FWD, timed)))
                return rc;
        } else {
            if ((rc = real_pass(bA, bB, true, timed))) return rc;
        }
        for (int j = 0; j < 3; ++j) out[j] = bB[j];
        return SPFC_OK;
    }

    // Ghost start (eq. scheme-SAV-initial-1): phi^{-1} into the other slot, r^0 and r^{-1}.
    int ghost(double dt) {
        int rc;
        const int o = 1 - ctx->slotX;
        char* X = ctx->slot(ctx->slotX);
        if ((rc = spec_inv(X, X, nullptr, Pending{}, 1.0, 0.0, true, false))) return rc;
        char* fl[3];
        if ((rc = flux(false, fl))) return rc;
        if ((rc = spec_fwd(fl, X, X, FWD_GHOST, ctx->slot(o), 1.0, 0.0, 0.0, dt, 1.0, 0.0, false))) return rc;
        if ((rc = finalize(FIN_GHOST_R0, ctx->sh.A.grid, 0))) return rc;
        if ((rc = e1_pass(ctx->slot(o), ctx->slot(o), FIN_GHOST_RM1))) return rc;
        ctx->slotY = o;
        return SPFC_OK;
    }

    // One step: (pending update, closing that step), gradient and inverse passes,
    // real-space pass, forward pass + N + inner products; leaves this step pending.
    // f^{n+1} of the next step into force_buf from its terms and coefficients coef[terms]
    int force(const double* coef) {
        ForceArgs<T> f{};
        f.out = (C*)ctx->force_buf;
        f.g = (const C*)(ctx->force_buf + ctx->lay.F);
        f.terms = ctx->force_terms;
        f.coef = coef;
        f.total = (long long)ctx->lay.fs;
        CK(Kern<T>::force(f, ctx->stream));
        return SPFC_OK;
    }

    // coef (device, or null): forcing coefficients of this step
    int body(Pending& pend, double dt, double a0, double a1, double a2, double e1, double e2, int check,
             bool timed, const double* coef = nullptr) {
        int rc;
        if (!pend.open) {
            if ((rc = spec_inv(ctx->slot(ctx->slotX), ctx->slot(ctx->slotY), nullptr, pend, e1, e2, true, timed)))
                return rc;
        } else {
            const int target = ctx->slotY != ctx->slotX ? ctx->slotY : 1 - ctx->slotX;
            if ((rc = spec_inv(ctx->slot(ctx->slotX), ctx->slot(ctx->slotY), ctx->slot(target), pend, e1, e2, true,
                               timed)))
                return rc;
            ctx->slotY = ctx->slotX;
            ctx->slotX = target;
            ctx->step += 1;
        }
        // the pending step's forcing has been read by the update above: now this step's
        if (coef && (rc = force(coef))) return rc;
        char* fl[3];
        if ((rc = flux(timed, fl))) return rc;
        if ((rc = spec_fwd(fl, ctx->slot(ctx->slotX), ctx->slot(ctx->slotY), coef ? FWD_SOLVE_FORCED : FWD_SOLVE,
                           nullptr, a0, a1, a2, dt, e1, e2, timed, coef ? ctx->force_buf : nullptr)))
            return rc;
        pend.forced = coef != nullptr;
        pend.open = true;
        pend.a0 = a0;
        pend.a1 = a1;
        pend.a2 = a2;
        pend.dt = dt;
        pend.check = check;
        if (!ctx->fin_in) {
            // the SAV scalar: xi, r^{n+1}, the record of phi^n
            if ((rc = finalize(FIN_STEP, 0, 0, &pend, timed))) return rc;
        }
        return SPFC_OK;
    }

    // `pairs` replays of a graph of two steady steps.  The launches of two steps
    // depend only on dt, the slot pair and the scalar-block parity, and two steps
    // bring all three back; a graph is captured on first use of such a key and
    // kept (the last few keys).
    int graph_pairs(Pending& pend, double dt, int64_t pairs) {
        const auto key = std::make_tuple(dt, ctx->slotX, ctx->slotY, ctx->cur_sc);
        hipGraphExec_t exec = nullptr;
        for (auto& g : ctx->graphs)
            if (g.first == key) exec = g.second;
        if (!exec) {
            const int sx = ctx->slotX, sy = ctx->slotY, cs = ctx->cur_sc;
            const int64_t st = ctx->step;
            const Pending p0 = pend;
            CK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
            int rc = SPFC_OK;
            for (int k = 0; k < 2 && rc == SPFC_OK; ++k) rc = body(pend, dt, kA0, kA1, kA2, kE1, kE2, 1, false);
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(ctx->stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            CK(ec);
            const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            CK(ei);
            if (ctx->graphs.size() >= 4) {
                (void)hipGraphExecDestroy(ctx->graphs.front().second);
                ctx->graphs.erase(ctx->graphs.begin());
            }
            ctx->graphs.push_back({key, exec});
            // capture only recorded the launches: back to the state before them
            ctx->slotX = sx;
            ctx->slotY = sy;
            ctx->cur_sc = cs;
            ctx->step = st;
            pend = p0;
        }
        for (int64_t i = 0; i < pairs; ++i) CK(hipGraphLaunch(exec, ctx->stream));
        ctx->step += 2 * pairs;
        return SPFC_OK;
    }

    // A call of n steps of size dt in phases: run_begin (restart at a new dt or at the
    // start), run_one per step (or graph replays of steady pairs), run_end (the last
    // update and the record of the state it reaches).
    int run_begin(StepRun& s, double dt) {
        int rc;
        s = StepRun{};
        s.restart = !ctx->started || dt != ctx->dt_prev;
        if (s.restart) {
            if (ctx->step == 0 && !ctx->started && ctx->prm.startup == SPFC_STARTUP_GHOST) {
                if ((rc = ghost(dt))) return rc;
            } else {
                // phi^{-1} = phi^0, r^{-1} = r^0 = sqrt(E_1(phi^0))
                ctx->slotY = ctx->slotX;
                if ((rc = e1_pass(ctx->slot(ctx->slotX), ctx->slot(ctx->slotX), FIN_RESTART))) return rc;
                s.first_order = (ctx->step == 0 && !ctx->started && ctx->prm.startup == SPFC_STARTUP_SAV1);
            }
        }
        return SPFC_OK;
    }

    // a pending BDF2 step of this dt whose rise check is on, two distinct slots: the
    // next two steps then launch what the two before them did
    bool run_steady(const StepRun& s, double dt) const {
        const Pending& p = s.pend;
        return p.open && p.a0 == kA0 && p.check == 1 && p.dt == dt && !p.forced && ctx->slotX != ctx->slotY;
    }

    // coef (device, force_terms values, or null): the forcing coefficients of this step
    int run_one(StepRun& s, double dt, const double* coef) {
        const bool sav1 = s.first_order && s.i == 0;
        const int check = (s.i == 0 && s.restart) ? 0 : 1;
        const bool timed = s.i >= ctx->timed_from;
        int rc;
        if (sav1) rc = body(s.pend, dt, 1.0, 1.0, 0.0, 1.0, 0.0, check, timed, coef);
        else rc = body(s.pend, dt, kA0, kA1, kA2, kE1, kE2, check, timed, coef);
        if (rc) return rc;
        ++s.i;
        return SPFC_OK;
    }

    // The launches of two steady steps (for a capture; the caller restores the state).
    int steady_pair(StepRun& s, double dt) {
        int rc = SPFC_OK;
        for (int k = 0; k < 2 && rc == SPFC_OK; ++k) rc = body(s.pend, dt, kA0, kA1, kA2, kE1, kE2, 1, false);
        return rc;
    }

    // n steps of size dt; coef (device, n x force_terms, or null): the forcing
    // coefficients of each step (its f^{n+1})
    int steps(double dt, int64_t n, const double* coef = nullptr) {
        int rc;
        StepRun s;
        if ((rc = run_begin(s, dt))) return rc;
        const bool graphs = ctx->use_graph && !ctx->profiling && ctx->stream != nullptr && !coef;
        while (s.i < n) {
            if (graphs && run_steady(s, dt) && n - s.i >= 2) {
                const int64_t pairs = (n - s.i) / 2;
                if ((rc = graph_pairs(s.pend, dt, pairs))) return rc;
                s.i += 2 * pairs;
                continue;
            }
            if ((rc = run_one(s, dt, coef ? coef + s.i * ctx->force_terms : nullptr))) return rc;
        }
        return run_end(s, dt);
    }

    // apply the last update and record the state it reaches
    int run_end(StepRun& s, double dt) {
        int rc;
        const Pending& pend = s.pend;
        const int target = ctx->slotY != ctx->slotX ? ctx->slotY : 1 - ctx->slotX;
        UpdateArgs<T> u{};
        u.cur = (const C*)ctx->slot(ctx->slotX);
        u.prev = (const C*)ctx->slot(ctx->slotY);
        u.nhat = (const C*)ctx->nhat();
        u.out_new = (C*)ctx->slot(target);
        u.total = (long long)ctx->lay.fs;
        u.NL = ctx->nl();
        u.B = ctx->lineB();
        u.ua0 = pend.a0;
        u.ua1 = pend.a1;
        u.ua2 = pend.a2;
        u.udt = pend.dt;
        u.fin = ctx->fin_in ? 1 : 0;
        u.fi = finish_in(pend.check);
        u.part = ctx->partQ();
        u.fs = ctx->lay.fs;
        u.geos = ctx->dgeos();
        u.fhat = pend.forced ? (const C*)ctx->force_buf : nullptr;
        CK(Kern<T>::update(ctx->sz.dim, ctx->stab, u, ctx->sh.updGrid, ctx->M, 256, ctx->stream));
        if (u.fin) ctx->cur_sc = 1 - ctx->cur_sc;
        ctx->slotY = ctx->slotX;
        ctx->slotX = target;
        ctx->step += 1;
        if ((rc = finalize(FIN_STATE, ctx->sh.updGrid, 1, nullptr, false, dt))) return rc;
        ctx->started = true;
        ctx->dt_prev = dt;
        return SPFC_OK;
    }

    // Real fields (doubles, x fastest) of members m0 .. m0 + count - 1 -> their half
    // spectra at dst (a field region laid out like a slot); real[j] is member m0 + j's field.  One launch per pass for up
    // to ROW_TAB members.
    int forward_real(const double* const* real, int m0, int count, char* dst) {
        for (int c0 = 0; c0 < count; c0 += ROW_TAB) {
            const int cn = std::min(ROW_TAB, count - c0);
            const size_t mo = ctx->moff(m0 + c0);
            RowArgs<T> r{};
            r.spec = (C*)(ctx->bufA(0) + mo);
            r.fs = ctx->lay.fs;
            r.tw = (const C*)ctx->tw();
            r.tws = ctx->lay.ntab / ctx->sz.nx;
            r.nrows = ctx->sz.ny * ctx->sz.nz;
            r.G = ctx->sh.r2c.G;
            r.scale = 1.0;
            for (int j = 0; j < cn; ++j) r.real[j] = const_cast<double*>(real[c0 + j]);
            LaunchShape rs = ctx->sh.r2c;
            rs.members = cn;
            CK(Kern<T>::r2c_rows(ctx->sz.nx, r, rs, ctx->stream));
        }
        PassArgs<T> p{};
        p.tw = (const C*)ctx->tw();
        p.fs = ctx->lay.fs;
        const size_t mo = ctx->moff(m0);
        if (ctx->sz.dim == 3) {
            // [X][Z][Y] -> transform y -> [X][Y][Z]
            p.in[0] = (const C*)(ctx->bufA(0) + mo);
            p.out[0] = (C*)(ctx->bufB(0) + mo);
            p.tws = ctx->lay.ntab / ctx->sz.ny;
            p.nlines = ctx->sz.nxh * ctx->sz.nz;
            p.B = ctx->sz.nz;
            p.G = ctx->sh.swapInit.G;
            LaunchShape ss = ctx->sh.swapInit;
            ss.members = count;
            CK(Kern<T>::pass(ctx->sz.ny, -1, OUT_SWAP, 1, p, ss, ctx->stream));
            p.in[0] = (const C*)(ctx->bufB(0) + mo);
        } else {
            p.in[0] = (const C*)(ctx->bufA(0) + mo);
        }
        p.out[0] = (C*)(dst + mo);
        p.tws = ctx->lay.ntab / ctx->nl();
        p.nlines = ctx->nlines();
        p.B = ctx->lineB();
        p.G = ctx->sh.keep.G;
        LaunchShape ks = ctx->sh.keep;
        ks.members = count;
        CK(Kern<T>::pass(ctx->nl(), -1, OUT_KEEP, 1, p, ks, ctx->stream));
        return SPFC_OK;
    }

    // half spectra of members m0 .. m0 + count - 1's newest state -> real fields out[j]
    int inverse_real(int m0, int count, void* const* out, bool out_fp32) {
        const size_t mo = ctx->moff(m0);
        PassArgs<T> p{};
        p.tw = (const C*)ctx->tw();
        p.fs = ctx->lay.fs;
        p.in[0] = (const C*)(ctx->slot(ctx->slotX) + mo);
        p.out[0] = (C*)(ctx->bufA(0) + mo);
        p.tws = ctx->lay.ntab / ctx->nl();
        p.nlines = ctx->nlines();
        p.B = ctx->lineB();
        p.G = ctx->sh.rot.G;
        LaunchShape rs = ctx->sh.rot;
        rs.members = count;
        CK(Kern<T>::pass(ctx->nl(), +1, OUT_ROTATE, 1, p, rs, ctx->stream));
        char* rows = ctx->bufA(0);
        if (ctx->sz.dim == 3) {
            // [Z][X][Y] -> transform y -> [Z][Y][X]
            p.in[0] = (const C*)(ctx->bufA(0) + mo);
            p.out[0] = (C*)(ctx->bufB(0) + mo);
            p.tws = ctx->lay.ntab / ctx->sz.ny;
            p.nlines = ctx->sz.nz * ctx->sz.nxh;
            p.B = ctx->sz.nxh;
            p.G = ctx->sh.swapGet.G;
            LaunchShape ss = ctx->sh.swapGet;
            ss.members = count;
            CK(Kern<T>::pass(ctx->sz.ny, +1, OUT_SWAP, 1, p, ss, ctx->stream));
            rows = ctx->bufB(0);
        }
        for (int c0 = 0; c0 < count; c0 += ROW_TAB) {
            const int cn = std::min(ROW_TAB, count - c0);
            RowArgs<T> r{};
            r.spec = (C*)(rows + ctx->moff(m0 + c0));
            r.fs = ctx->lay.fs;
            r.tw = (const C*)ctx->tw();
            r.tws = ctx->lay.ntab / ctx->sz.nx;
            r.nrows = ctx->sz.ny * ctx->sz.nz;
            r.G = ctx->sh.c2r.G;
            r.scale = ctx->geos[m0].inv_npts;   // one grid size per class
            for (int j = 0; j < cn; ++j) r.real[j] = out[c0 + j];
            LaunchShape cs = ctx->sh.c2r;
            cs.members = cn;
            CK(Kern<T>::c2r_rows(ctx->sz.nx, out_fp32, r, cs, ctx->stream));
        }
        return SPFC_OK;
    }

    // twiddle table and the members' geometry
    int write_tables() {
        const int n = ctx->lay.ntab;
        std::vector<C> h(n);
        for (int j = 0; j < n; ++j) {
            const long double ang = -2.0L * 3.141592653589793238462643383279502884L * (long double)j / (long double)n;
            h[j] = mk<T>(T(cosl(ang)), T(sinl(ang)));
        }
        CK(hipMemcpyAsync(ctx->tw(), h.data(), n * sizeof(C), hipMemcpyHostToDevice, ctx->stream));
        CK(hipMemcpyAsync(ctx->ws + ctx->lay.off_geo, ctx->geos.data(), ctx->M * sizeof(Geo), hipMemcpyHostToDevice,
                          ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        return SPFC_OK;
    }
};

template <typename F>
int with_pipe(spfc_ctx* ctx, F&& f) {
    if (ctx->prm.precision == SPFC_FP32) {
        Pipe<float> p{ctx};
        return f(p);
    }
    Pipe<double> p{ctx};
    return f(p);
}

// host copy of a device field; SPFC_E_INVAL if any value is not finite
int check_finite_field(const double* dev, size_t n, hipStream_t stream) {
    std::vector<double> host(n);
    if (hipMemcpyAsync(host.data(), dev, n * sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return SPFC_E_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return SPFC_E_DEVICE;
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return SPFC_E_INVAL;
    return SPFC_OK;
}

size_t class_bytes(const spfc_grid& g, const spfc_params& p, int M) {
    const Sizes s = sizes_of(g, p.precision);
    return layout_of(s, p.history, M).total;
}

// Context over workspace `ws` for members idx[0..M) of (grids, params, phi0): same
// sizes and precision.  Transforms the initial fields and computes r^0.
int make_ctx(const spfc_grid* grids, const spfc_params* params, const int* idx, int M, const double* const* phi0,
             char* ws, hipStream_t stream, spfc_ctx** out) {
    const spfc_params& p0 = params[idx[0]];
    spfc_ctx* ctx = new (std::nothrow) spfc_ctx();
    if (!ctx) return SPFC_E_NOMEM;
    ctx->prm = p0;
    ctx->M = M;
    ctx->stab = false;
    bool beta = false;
    for (int m = 0; m < M; ++m) {
        ctx->geos.push_back(make_geo(grids[idx[m]], params[idx[m]]));
        ctx->stab = ctx->stab || params[idx[m]].stab != 0.0;
        beta = beta || params[idx[m]].beta != 0.0;
    }
    ctx->sz = sizes_of(grids[idx[0]], p0.precision);
    ctx->sz.beta = beta;   // some member has the quartic term: the class runs that variant
    ctx->plan = tune_plan(ctx->sz.dim);
    if (!plan_fits(ctx->sz, M, ctx->plan, device_lds_max())) {
        delete ctx;
        return SPFC_E_INVAL;
    }
    ctx->sh = shapes_of(ctx->sz, M, ctx->plan);
    ctx->lay = layout_of(ctx->sz, p0.history, M);
    ctx->stream = stream;
    ctx->ws = ws;
    ctx->slotX = ctx->slotY = 0;
    ctx->step = 0;
    ctx->dt_prev = 0.0;
    ctx->started = false;
    ctx->broken = false;
    ctx->energy_tol = p0.energy_tol > 0 ? p0.energy_tol : (p0.precision == SPFC_FP32 ? 1e-6 : 1e-12);
    ctx->cur_sc = 0;
    set_plan(ctx, ctx->plan);
    ctx->use_graph = false;
    ctx->profiling = false;
    ctx->reps = 1;
    ctx->timed_from = 0;
    for (int i = 0; i < R_COUNT; ++i) {
        ctx->role_ms[i] = 0;
        ctx->role_n[i] = 0;
    }
    const Layout& lay = ctx->lay;
    int rc = SPFC_OK;
    // scalar blocks (step_x = 0, flags clear) and history start at zero
    if (hipMemsetAsync(ws + lay.off_sc, 0, lay.total - lay.off_sc, stream) != hipSuccess) rc = SPFC_E_DEVICE;
    if (!rc)
        rc = with_pipe(ctx, [&](auto& p) {
            int r;
            if ((r = p.write_tables())) return r;
            std::vector<const double*> in(M);
            for (int m = 0; m < M; ++m) in[m] = phi0[idx[m]];
            if ((r = p.forward_real(in.data(), 0, M, ctx->slot(0)))) return r;
            // r^0 = sqrt(E_1(phi^0)) (after eq. scheme-SAV-initial-1)
            return p.e1_pass(ctx->slot(0), ctx->slot(0), FIN_RESTART);
        });
    if (!rc && hipStreamSynchronize(stream) != hipSuccess) rc = SPFC_E_DEVICE;
    if (rc) {
        delete ctx;
        return rc;
    }
    *out = ctx;
    return SPFC_OK;
}

// Start the run of every member of a class again from new fields (as at init): state
// from the fields, step 0, start-up mode on the next step, flags and history cleared.
int reset_ctx(spfc_ctx* ctx, const int* idx, const double* const* phi) {
    if (ctx->broken) return SPFC_E_DEVICE;
    drop_graph(ctx);
    CK(hipMemsetAsync(ctx->ws + ctx->lay.off_sc, 0, ctx->lay.total - ctx->lay.off_sc, ctx->stream));
    ctx->slotX = ctx->slotY = 0;
    ctx->step = 0;
    ctx->dt_prev = 0.0;
    ctx->started = false;
    ctx->cur_sc = 0;
    int rc = with_pipe(ctx, [&](auto& p) {
        int r;
        std::vector<const double*> in(ctx->M);
        for (int m = 0; m < ctx->M; ++m) in[m] = phi[idx[m]];
        if ((r = p.forward_real(in.data(), 0, ctx->M, ctx->slot(0)))) return r;
        return p.e1_pass(ctx->slot(0), ctx->slot(0), FIN_RESTART);
    });
    if (rc) return rc;
    CK(hipStreamSynchronize(ctx->stream));
    return SPFC_OK;
}

void free_ctx(spfc_ctx* ctx) {
    if (!ctx->broken) (void)hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
    for (auto& u : ctx->ev_used) {
        (void)hipEventDestroy(u.a);
        (void)hipEventDestroy(u.b);
    }
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
}

int ctx_step(spfc_ctx* ctx, double dt, int64_t n) {
    if (ctx->broken) return SPFC_E_DEVICE;
    if (n == 0) return SPFC_OK;
    return with_pipe(ctx, [&](auto& p) { return p.steps(dt, n); });
}

// Every class stream waits for the work queued on the batch's stream so far.
int batch_fork(spfc_batch* b) {
    if (hipEventRecord(b->fork, b->stream) != hipSuccess) return SPFC_E_DEVICE;
    int rc = SPFC_OK;
    for (auto s : b->cstream)
        if (hipStreamWaitEvent(s, b->fork, 0) != hipSuccess) rc = SPFC_E_DEVICE;
    return rc;
}

// The batch's stream waits for the work queued on every class stream so far.
int batch_join(spfc_batch* b) {
    int rc = SPFC_OK;
    for (size_t c = 0; c < b->cstream.size(); ++c)
        if (hipEventRecord(b->join[c], b->cstream[c]) != hipSuccess ||
            hipStreamWaitEvent(b->stream, b->join[c], 0) != hipSuccess)
            rc = SPFC_E_DEVICE;
    return rc;
}

// `pairs` replays, on the batch's stream, of one graph holding two steady steps of every
// class (each class a branch forked from and joined back into the batch's stream), so
// the whole batch advances two steps per graph launch.  Captured on first use of its key
// (the class states the two steps depend on) and kept (the last few keys).  Called with
// the class streams forked from the batch's stream; they are forked again after the
// replays.
int batch_graph_pairs(spfc_batch* b, std::vector<StepRun>& runs, double dt, int64_t pairs) {
    const size_t nc = b->cls.size();
    std::vector<int64_t> key;
    int64_t dbits = 0;
    std::memcpy(&dbits, &dt, sizeof(dbits));
    key.push_back(dbits);
    for (auto* c : b->cls) {
        key.push_back(c->slotX);
        key.push_back(c->slotY);
        key.push_back(c->cur_sc);
        key.push_back(c->graph_gen);
    }
    hipGraphExec_t exec = nullptr;
    for (auto& g : b->graphs)
        if (g.first == key) exec = g.second;
    // the replays follow what the class streams hold so far
    int rc = batch_join(b);
    if (rc) return rc;
    if (!exec) {
        struct Saved {
            int sx, sy, cs;
            int64_t st;
            Pending pend;
        };
        std::vector<Saved> saved(nc);
        for (size_t c = 0; c < nc; ++c)
            saved[c] = {b->cls[c]->slotX, b->cls[c]->slotY, b->cls[c]->cur_sc, b->cls[c]->step, runs[c].pend};
        if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return SPFC_E_DEVICE;
        rc = batch_fork(b);
        for (size_t c = 0; c < nc && rc == SPFC_OK; ++c)
            rc = with_pipe(b->cls[c], [&](auto& p) { return p.steady_pair(runs[c], dt); });
        // join every branch before ending the capture, also after an error
        const int rj = batch_join(b);
        if (!rc) rc = rj;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->stream, &g);
        // capture only recorded the launches: back to the states before them
        for (size_t c = 0; c < nc; ++c) {
            b->cls[c]->slotX = saved[c].sx;
            b->cls[c]->slotY = saved[c].sy;
            b->cls[c]->cur_sc = saved[c].cs;
            b->cls[c]->step = saved[c].st;
            runs[c].pend = saved[c].pend;
        }
        if (rc || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : SPFC_E_DEVICE;
        }
        const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return SPFC_E_DEVICE;
        if (b->graphs.size() >= 4) {
            (void)hipGraphExecDestroy(b->graphs.front().second);
            b->graphs.erase(b->graphs.begin());
        }
        b->graphs.push_back({key, exec});
    }
    for (int64_t i = 0; i < pairs; ++i)
        if (hipGraphLaunch(exec, b->stream) != hipSuccess) return SPFC_E_DEVICE;
    for (size_t c = 0; c < nc; ++c) {
        b->cls[c]->step += 2 * pairs;
        runs[c].i += 2 * pairs;
    }
    return batch_fork(b);
}

// n steps of every class of a batch with class streams (forked already), replaying
// steady pairs of steps of the whole batch from one graph.
int batch_steps_graph(spfc_batch* b, double dt, int64_t n) {
    const size_t nc = b->cls.size();
    std::vector<StepRun> runs(nc);
    int rc;
    for (size_t c = 0; c < nc; ++c) {
        if (b->cls[c]->broken) return SPFC_E_DEVICE;
        if (b->cls[c]->profiling) {
            // profiling times each launch: direct launches, class by class
            for (auto* x : b->cls)
                if ((rc = ctx_step(x, dt, n))) return rc;
            return SPFC_OK;
        }
    }
    for (size_t c = 0; c < nc; ++c)
        if ((rc = with_pipe(b->cls[c], [&](auto& p) { return p.run_begin(runs[c], dt); }))) return rc;
    int64_t i = 0;
    while (i < n) {
        bool steady = n - i >= 2;
        for (size_t c = 0; c < nc && steady; ++c)
            steady = with_pipe(b->cls[c], [&](auto& p) { return p.run_steady(runs[c], dt) ? 1 : 0; }) == 1;
        if (steady) {
            const int64_t pairs = (n - i) / 2;
            if ((rc = batch_graph_pairs(b, runs, dt, pairs))) return rc;
            i += 2 * pairs;
            continue;
        }
        for (size_t c = 0; c < nc; ++c)
            if ((rc = with_pipe(b->cls[c], [&](auto& p) { return p.run_one(runs[c], dt, nullptr); }))) return rc;
        ++i;
    }
    for (size_t c = 0; c < nc; ++c)
        if ((rc = with_pipe(b->cls[c], [&](auto& p) { return p.run_end(runs[c], dt); }))) return rc;
    return SPFC_OK;
}

int ctx_status(spfc_ctx* ctx, int m, uint32_t* flags) {
    if (ctx->broken) return SPFC_E_DEVICE;
    unsigned int f = 0;
    CK(hipMemcpyAsync(&f, &ctx->sc(m)->flags, sizeof(f), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    *flags = f;
    return SPFC_OK;
}

int ctx_mass(spfc_ctx* ctx, int m, double* mean) {
    if (ctx->broken) return SPFC_E_DEVICE;
    const char* src = ctx->slot(ctx->slotX) + ctx->moff(m);
    double re = 0.0;
    if (ctx->prm.precision == SPFC_FP32) {
        float v[2];
        CK(hipMemcpyAsync(v, src, sizeof(v), hipMemcpyDeviceToHost, ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        re = v[0];
    } else {
        double v[2];
        CK(hipMemcpyAsync(v, src, sizeof(v), hipMemcpyDeviceToHost, ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        re = v[0];
    }
    *mean = re * ctx->geos[m].inv_npts;
    return SPFC_OK;
}

// the query pass covers every member of the context; member m's values are read back
int ctx_energy(spfc_ctx* ctx, int m, spfc_energy_t* out) {
    if (ctx->broken) return SPFC_E_DEVICE;
    int rc = with_pipe(ctx, [&](auto& p) {
        return p.e1_pass(ctx->slot(ctx->slotX), ctx->slot(ctx->slotY), FIN_QUERY);
    });
    if (rc) return rc;
    DevScalars sc;
    CK(hipMemcpyAsync(&sc, ctx->sc(m), sizeof(sc), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    const Geo& g = ctx->geos[m];
    const double rn = sc.r_n, rm = sc.r_nm1;
    out->modified_energy = 0.25 * (sc.q_norm[0] + sc.q_norm[1]) + 0.5 * (rn * rn + (2 * rn - rm) * (2 * rn - rm)) +
                           0.25 * g.stab * ctx->dt_prev * sc.q_norm[4];
    out->E1 = sc.q_E1;
    out->energy = sc.q_E1 - g.e1_const + 0.5 * g.a * sc.q_norm[2] + 0.5 * sc.q_norm[3];
    out->sav_energy = 0.5 * g.a * sc.q_norm[2] + 0.5 * sc.q_norm[3] + rn * rn;
    out->r = rn;
    out->mean = sc.mean;
    out->step = ctx->step;
    return (sc.flags & SPFC_FLAG_NONFINITE) ? SPFC_E_NONFINITE : SPFC_OK;
}

int ctx_history(spfc_ctx* ctx, int m, int64_t first, int64_t count, spfc_record* out) {
    if (ctx->broken) return SPFC_E_DEVICE;
    if (count == 0) return SPFC_OK;
    const int64_t cap = ctx->prm.history;
    const int64_t last = first + count - 1;
    if (last > ctx->step || first < ctx->step + 1 - cap) return SPFC_E_STATE;
    static_assert(sizeof(Record) == sizeof(spfc_record), "record layout");
    CK(hipStreamSynchronize(ctx->stream));
    for (int64_t i = first; i <= last;) {
        const int64_t s = i % cap;
        const int64_t run = std::min<int64_t>(last - i + 1, cap - s);
        CK(hipMemcpy(out + (i - first), ctx->hist(m) + s, run * sizeof(Record), hipMemcpyDeviceToHost));
        i += run;
    }
    return SPFC_OK;
}

int ctx_get_phi(spfc_ctx* ctx, int m, void* out_dev, int dtype) {
    if (ctx->broken) return SPFC_E_DEVICE;
    void* out[1] = {out_dev};
    return with_pipe(ctx, [&](auto& p) { return p.inverse_real(m, 1, out, dtype == SPFC_FP32); });
}

// members grouped by (dim, n, precision), classes in order of first appearance
std::vector<std::vector<int>> group_members(int count, const spfc_grid* grids, const spfc_params* params) {
    std::map<std::tuple<int, int, int, int, int>, int> cls;
    std::vector<std::vector<int>> out;
    for (int i = 0; i < count; ++i) {
        const auto key = std::make_tuple(grids[i].dim, grids[i].n[0], grids[i].n[1],
                                         grids[i].dim == 3 ? grids[i].n[2] : 1, params[i].precision);
        auto it = cls.find(key);
        if (it == cls.end()) {
            cls.emplace(key, (int)out.size());
            out.push_back({i});
        } else {
            out[it->second].push_back(i);
        }
    }
    return out;
}

int validate_batch(int count, const spfc_grid* grids, const spfc_params* params) {
    if (count < 1 || !grids || !params) return SPFC_E_INVAL;
    for (int i = 0; i < count; ++i) {
        const int rc = validate(&grids[i], &params[i]);
        if (rc) return rc;
        if (params[i].startup != params[0].startup || params[i].history != params[0].history ||
            params[i].energy_tol != params[0].energy_tol)
            return SPFC_E_INVAL;
    }
    return SPFC_OK;
}

size_t batch_bytes(const std::vector<std::vector<int>>& classes, const spfc_grid* grids,
                   const spfc_params* params) {
    size_t total = 0;
    for (const auto& c : classes) total += class_bytes(grids[c[0]], params[c[0]], (int)c.size());
    return total;
}

bool member_ok(const spfc_batch* b, int member) { return b && member >= 0 && member < (int)b->where.size(); }

// ---------------------------------------------------------------- launch-plan tuner

// Run state of a context between calls: both state slots, both scalar-block copies
// and the history ring on the device (two contiguous ranges of the workspace),
// slot / step bookkeeping on the host.
struct HostState {
    int slotX, slotY, cur_sc;
    int64_t step;
    double dt_prev;
    bool started;
};

size_t snapshot_bytes(const spfc_ctx* ctx) {
    return 2 * ctx->lay.field_bytes + (ctx->lay.total - ctx->lay.off_sc);
}

int snapshot(spfc_ctx* ctx, char* dst, HostState& hs) {
    hs = {ctx->slotX, ctx->slotY, ctx->cur_sc, ctx->step, ctx->dt_prev, ctx->started};
    const size_t a = 2 * ctx->lay.field_bytes, b = ctx->lay.total - ctx->lay.off_sc;
    CK(hipMemcpyAsync(dst, ctx->slot(0), a, hipMemcpyDeviceToDevice, ctx->stream));
    CK(hipMemcpyAsync(dst + a, ctx->ws + ctx->lay.off_sc, b, hipMemcpyDeviceToDevice, ctx->stream));
    return SPFC_OK;
}

int restore(spfc_ctx* ctx, const char* src, const HostState& hs) {
    const size_t a = 2 * ctx->lay.field_bytes, b = ctx->lay.total - ctx->lay.off_sc;
    CK(hipMemcpyAsync(ctx->slot(0), src, a, hipMemcpyDeviceToDevice, ctx->stream));
    CK(hipMemcpyAsync(ctx->ws + ctx->lay.off_sc, src + a, b, hipMemcpyDeviceToDevice, ctx->stream));
    ctx->slotX = hs.slotX;
    ctx->slotY = hs.slotY;
    ctx->cur_sc = hs.cur_sc;
    ctx->step = hs.step;
    ctx->dt_prev = hs.dt_prev;
    ctx->started = hs.started;
    return SPFC_OK;
}

// Milliseconds of `trial` steps of size dt under plan tp, from the snapshot (after
// two untimed steps that absorb any restart): the smaller of two such timings, so that
// one disturbed timing does not decide a choice.
int time_plan(spfc_ctx* ctx, const TunePlan& tp, double dt, int64_t trial, const char* snap, const HostState& hs,
              hipEvent_t e0, hipEvent_t e1, float* ms) {
    set_plan(ctx, tp);
    int rc;
    float best = 0.f;
    for (int k = 0; k < 2; ++k) {
        if ((rc = restore(ctx, snap, hs))) return rc;
        if ((rc = ctx_step(ctx, dt, 2))) return rc;
        CK(hipEventRecord(e0, ctx->stream));
        if ((rc = ctx_step(ctx, dt, trial))) return rc;
        CK(hipEventRecord(e1, ctx->stream));
        CK(hipEventSynchronize(e1));
        float t = 0.f;
        CK(hipEventElapsedTime(&t, e0, e1));
        best = k == 0 ? t : std::min(best, t);
    }
    *ms = best;
    return SPFC_OK;
}

// Coordinate search over the values per thread (4, 8, 16) and workgroup size (128,
// 256 threads) of each step kernel, one kernel at a time, keeping a change only if
// it saves at least 2 %.  The run state is restored afterwards: tuning changes
// nothing but the plan (and with it the rounding of the transforms).
int tune_ctx(spfc_ctx* ctx, double dt, int64_t trial, char* snap) {
    HostState hs;
    int rc;
    if ((rc = snapshot(ctx, snap, hs))) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        ctx->broken = true;
        return SPFC_E_DEVICE;
    }
    TunePlan best = ctx->plan;
    float best_ms = 0.f;
    rc = time_plan(ctx, best, dt, trial, snap, hs, e0, e1, &best_ms);
    const size_t lds_max = device_lds_max();
    RolePlan TunePlan::*roles[4] = {&TunePlan::inv, &TunePlan::real, &TunePlan::fwd, &TunePlan::mid};
    const int nroles = ctx->sz.dim == 3 ? 4 : 3;
    for (int r = 0; r < nroles && !rc; ++r) {
        const int tmax = role_t_max(r, ctx->sz.dim);
        for (int E : {4, 8, 16}) {
            for (int T : {128, 256, 512}) {
                if (T > tmax) continue;
                TunePlan cand = best;
                if ((cand.*roles[r]).E == E && (cand.*roles[r]).T == T) continue;
                (cand.*roles[r]).E = E;
                (cand.*roles[r]).T = T;
                if (!plan_fits(ctx->sz, ctx->M, cand, lds_max)) continue;
                float ms = 0.f;
                if ((rc = time_plan(ctx, cand, dt, trial, snap, hs, e0, e1, &ms))) break;
                if (ms < 0.98f * best_ms) {
                    best = cand;
                    best_ms = ms;
                }
            }
            if (rc) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    set_plan(ctx, best);
    if ((rc = restore(ctx, snap, hs))) return rc;
    CK(hipStreamSynchronize(ctx->stream));
    return SPFC_OK;
}

// Per-launch duration of each step kernel in a steady step: from a snapshot, one
// untimed step, then one step in which every kernel is launched `reps` times back
// to back between two events (repeats of the update kernel overwrite the older
// state, so the run state is restored from the snapshot afterwards).
int time_ctx(spfc_ctx* ctx, double dt, int reps, char* snap) {
    HostState hs;
    int rc;
    if ((rc = snapshot(ctx, snap, hs))) return rc;
    if ((rc = drain_events(ctx))) return rc;
    const bool was = ctx->profiling;
    for (int i = 0; i < R_COUNT; ++i) {
        ctx->role_ms[i] = 0;
        ctx->role_n[i] = 0;
    }
    if ((rc = ctx_step(ctx, dt, 2))) return rc;   // steady, same dt
    ctx->profiling = true;
    ctx->reps = reps;
    ctx->timed_from = 1;
    rc = ctx_step(ctx, dt, 2);
    ctx->profiling = was;
    ctx->reps = 1;
    ctx->timed_from = 0;
    if (rc) return rc;
    if ((rc = drain_events(ctx))) return rc;
    if ((rc = restore(ctx, snap, hs))) return rc;
    CK(hipStreamSynchronize(ctx->stream));
    return SPFC_OK;
}

// values per thread and threads per workgroup the step kernels actually use
void get_plan(const spfc_ctx* ctx, int* out) {
    const LaunchShape* sh[4] = {&ctx->sh.A, &ctx->sh.B, &ctx->sh.Cf, &ctx->sh.midI};
    for (int i = 0; i < 4; ++i) {
        const bool used = i < 3 || ctx->sz.dim == 3;
        out[2 * i] = used ? sh[i]->E : 0;
        out[2 * i + 1] = used ? sh[i]->block : 0;
    }
}

}  // namespace

// ==================================================================== C ABI

extern "C" {

const char* spfc_strerror(int status) {
    switch (status) {
        case SPFC_OK: return "ok";
        case SPFC_E_INVAL: return "invalid argument";
        case SPFC_E_NOMEM: return "workspace too small";
        case SPFC_E_DEVICE: return "HIP device error";
        case SPFC_E_NONFINITE: return "non-finite value detected";
        case SPFC_E_STATE: return "call out of order or bad checkpoint";
        default: return "unknown status";
    }
}

int spfc_workspace_bytes(const spfc_grid* grid, const spfc_params* params, size_t* bytes) {
    if (!bytes) return SPFC_E_INVAL;
    const int rc = validate(grid, params);
    if (rc) return rc;
    *bytes = class_bytes(*grid, *params, 1);
    return SPFC_OK;
}

int spfc_init(const spfc_grid* grid, const spfc_params* params, const double* phi0_dev, void* workspace_dev,
              size_t workspace_bytes, void* hip_stream, spfc_ctx** out) {
    const TraceRange trace_("spfc_init");
    if (!out || !phi0_dev || !workspace_dev) return SPFC_E_INVAL;
    int rc = validate(grid, params);
    if (rc) return rc;
    if (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign) return SPFC_E_INVAL;
    if (workspace_bytes < class_bytes(*grid, *params, 1)) return SPFC_E_NOMEM;
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    const Sizes s = sizes_of(*grid, params->precision);
    if ((rc = check_finite_field(phi0_dev, (size_t)s.nx * s.ny * s.nz, stream))) return rc;
    const int idx = 0;
    return make_ctx(grid, params, &idx, 1, &phi0_dev, reinterpret_cast<char*>(workspace_dev), stream, out);
}

int spfc_step(spfc_ctx* ctx, double dt, int64_t n) {
    const TraceRange trace_("spfc_step");
    if (!ctx) return SPFC_E_INVAL;
    if (!(dt > 0.0) || !std::isfinite(dt) || n < 0) return SPFC_E_INVAL;
    return ctx_step(ctx, dt, n);
}

int spfc_forcing_bytes(spfc_ctx* ctx, int terms, size_t* bytes) {
    if (!ctx || !bytes || terms < 1 || terms > SPFC_MAX_FORCING_TERMS) return SPFC_E_INVAL;
    *bytes = (size_t)(terms + 1) * ctx->lay.F;
    return SPFC_OK;
}

int spfc_set_forcing(spfc_ctx* ctx, int terms, const double* const* g_dev, void* buf_dev, size_t bytes) {
    const TraceRange trace_("spfc_set_forcing");
    if (!ctx) return SPFC_E_INVAL;
    if (ctx->broken) return SPFC_E_DEVICE;
    if (terms == 0) {
        ctx->force_buf = nullptr;
        ctx->force_terms = 0;
        return SPFC_OK;
    }
    size_t need = 0;
    if (spfc_forcing_bytes(ctx, terms, &need) != SPFC_OK || !g_dev || !buf_dev || bytes < need ||
        (reinterpret_cast<uintptr_t>(buf_dev) & 255u) != 0)
        return SPFC_E_INVAL;
    for (int i = 0; i < terms; ++i)
        if (!g_dev[i]) return SPFC_E_INVAL;
    char* buf = static_cast<char*>(buf_dev);
    const int rc = with_pipe(ctx, [&](auto& p) -> int {
        int r;
        for (int i = 0; i < terms; ++i)
            if ((r = p.forward_real(&g_dev[i], 0, 1, buf + (size_t)(i + 1) * ctx->lay.F))) return r;
        return SPFC_OK;
    });
    if (rc) return rc;
    CK(hipStreamSynchronize(ctx->stream));
    ctx->force_buf = buf;
    ctx->force_terms = terms;
    return SPFC_OK;
}

int spfc_step_forced(spfc_ctx* ctx, double dt, int64_t n, const double* coef_dev) {
    const TraceRange trace_("spfc_step_forced");
    if (!ctx || !coef_dev || !ctx->force_buf) return SPFC_E_INVAL;
    if (!(dt > 0.0) || !std::isfinite(dt) || n < 0) return SPFC_E_INVAL;
    // the ghost start would need f^0 as well, and the forced kernels are the plain scheme's:
    // neither is offered with forcing
    if ((!ctx->started && ctx->prm.startup == SPFC_STARTUP_GHOST) || ctx->stab) return SPFC_E_INVAL;
    if (ctx->broken) return SPFC_E_DEVICE;
    if (n == 0) return SPFC_OK;
    return with_pipe(ctx, [&](auto& p) { return p.steps(dt, n, coef_dev); });
}

int spfc_set_graph(spfc_ctx* ctx, int enable) {
    if (!ctx) return SPFC_E_INVAL;
    ctx->use_graph = enable != 0;
    if (!ctx->use_graph) drop_graph(ctx);
    return SPFC_OK;
}

int spfc_step_count(spfc_ctx* ctx, int64_t* n) {
    if (!ctx || !n) return SPFC_E_INVAL;
    *n = ctx->step;
    return SPFC_OK;
}

int spfc_status(spfc_ctx* ctx, uint32_t* flags) {
    if (!ctx || !flags) return SPFC_E_INVAL;
    return ctx_status(ctx, 0, flags);
}

int spfc_mass(spfc_ctx* ctx, double* mean) {
    if (!ctx || !mean) return SPFC_E_INVAL;
    return ctx_mass(ctx, 0, mean);
}

int spfc_energy(spfc_ctx* ctx, spfc_energy_t* out) {
    const TraceRange trace_("spfc_energy");
    if (!ctx || !out) return SPFC_E_INVAL;
    return ctx_energy(ctx, 0, out);
}

int spfc_history(spfc_ctx* ctx, int64_t first, int64_t count, spfc_record* out) {
    const TraceRange trace_("spfc_history");
    if (!ctx || (!out && count > 0) || first < 0 || count < 0) return SPFC_E_INVAL;
    return ctx_history(ctx, 0, first, count, out);
}

int spfc_get_phi(spfc_ctx* ctx, void* out_dev, int dtype) {
    const TraceRange trace_("spfc_get_phi");
    if (!ctx || !out_dev || (dtype != SPFC_FP64 && dtype != SPFC_FP32)) return SPFC_E_INVAL;
    return ctx_get_phi(ctx, 0, out_dev, dtype);
}

int spfc_state_bytes(spfc_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return SPFC_E_INVAL;
    *bytes = align_up(sizeof(CkptHeader)) + 2 * align_up(ctx->lay.F);
    return SPFC_OK;
}

int spfc_save_state(spfc_ctx* ctx, void* out_dev, size_t bytes) {
    const TraceRange trace_("spfc_save_state");
    if (!ctx || !out_dev) return SPFC_E_INVAL;
    if (ctx->broken) return SPFC_E_DEVICE;
    size_t need = 0;
    spfc_state_bytes(ctx, &need);
    if (bytes < need) return SPFC_E_STATE;
    CkptHeader hd{};
    hd.magic = kMagic;
    hd.step = ctx->step;
    hd.dt_prev = ctx->dt_prev;
    hd.started = ctx->started ? 1 : 0;
    hd.slot_same = ctx->slotX == ctx->slotY ? 1 : 0;
    hd.prec = ctx->prm.precision;
    hd.dim = ctx->sz.dim;
    hd.n[0] = ctx->sz.nx;
    hd.n[1] = ctx->sz.ny;
    hd.n[2] = ctx->sz.nz;
    CK(hipMemcpyAsync(&hd.sc, ctx->sc(), sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    char* o = reinterpret_cast<char*>(out_dev);
    CK(hipMemcpyAsync(o, &hd, sizeof(hd), hipMemcpyHostToDevice, ctx->stream));
    const size_t off = align_up(sizeof(CkptHeader));
    CK(hipMemcpyAsync(o + off, ctx->slot(ctx->slotX), ctx->lay.F, hipMemcpyDeviceToDevice, ctx->stream));
    CK(hipMemcpyAsync(o + off + align_up(ctx->lay.F), ctx->slot(ctx->slotY), ctx->lay.F, hipMemcpyDeviceToDevice,
                      ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    return SPFC_OK;
}

int spfc_load_state(spfc_ctx* ctx, const void* in_dev, size_t bytes) {
    const TraceRange trace_("spfc_load_state");
    if (!ctx || !in_dev) return SPFC_E_INVAL;
    if (ctx->broken) return SPFC_E_DEVICE;
    size_t need = 0;
    spfc_state_bytes(ctx, &need);
    if (bytes < need) return SPFC_E_STATE;
    CkptHeader hd{};
    const char* in = reinterpret_cast<const char*>(in_dev);
    CK(hipMemcpyAsync(&hd, in, sizeof(hd), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    if (hd.magic != kMagic || hd.prec != ctx->prm.precision || hd.dim != ctx->sz.dim || hd.n[0] != ctx->sz.nx ||
        hd.n[1] != ctx->sz.ny || hd.n[2] != ctx->sz.nz)
        return SPFC_E_STATE;
    drop_graph(ctx);
    const size_t off = align_up(sizeof(CkptHeader));
    CK(hipMemcpyAsync(ctx->slot(0), in + off, ctx->lay.F, hipMemcpyDeviceToDevice, ctx->stream));
    if (!hd.slot_same)
        CK(hipMemcpyAsync(ctx->slot(1), in + off + align_up(ctx->lay.F), ctx->lay.F, hipMemcpyDeviceToDevice,
                          ctx->stream));
    ctx->cur_sc = 0;
    CK(hipMemcpyAsync(ctx->sc(), &hd.sc, sizeof(DevScalars), hipMemcpyHostToDevice, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    ctx->slotX = 0;
    ctx->slotY = hd.slot_same ? 0 : 1;
    ctx->step = hd.step;
    ctx->dt_prev = hd.dt_prev;
    ctx->started = hd.started != 0;
    return SPFC_OK;
}

int spfc_profile(spfc_ctx* ctx, int enable) {
    if (!ctx) return SPFC_E_INVAL;
    const int rc = drain_events(ctx);
    if (rc) return rc;
    ctx->profiling = enable != 0;
    if (enable) {
        for (int i = 0; i < R_COUNT; ++i) {
            ctx->role_ms[i] = 0;
            ctx->role_n[i] = 0;
        }
    }
    return SPFC_OK;
}

int spfc_kernel_times(spfc_ctx* ctx, int cap, const char** names, double* avg_ms, int64_t* launches,
                      double* bytes_per_launch, int* count) {
    if (!ctx || !count) return SPFC_E_INVAL;
    const int rc = drain_events(ctx);
    if (rc) return rc;
    const double F = (double)ctx->lay.F * ctx->M;
    const int d = ctx->sz.dim;
    const double bytes[R_COUNT] = {6.0 * F, 5.0 * F, 2.0 * d * F, 5.0 * F, 5.0 * F, 0.0};
    int k = 0;
    for (int i = 0; i < R_COUNT; ++i) {
        if (ctx->role_n[i] == 0) continue;
        if (k < cap) {
            if (names) names[k] = kRoleNames[i];
            if (avg_ms) avg_ms[k] = ctx->role_ms[i] / (double)ctx->role_n[i];
            if (launches) launches[k] = ctx->role_n[i];
            if (bytes_per_launch) bytes_per_launch[k] = bytes[i];
        }
        ++k;
    }
    *count = k;
    return SPFC_OK;
}

int spfc_tune_bytes(spfc_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return SPFC_E_INVAL;
    *bytes = snapshot_bytes(ctx);
    return SPFC_OK;
}

int spfc_tune(spfc_ctx* ctx, double dt, int64_t trial_steps, void* scratch_dev, size_t scratch_bytes) {
    const TraceRange trace_("spfc_tune");
    if (!ctx || !scratch_dev) return SPFC_E_INVAL;
    if (!(dt > 0.0) || !std::isfinite(dt) || trial_steps < 1) return SPFC_E_INVAL;
    if (scratch_bytes < snapshot_bytes(ctx)) return SPFC_E_NOMEM;
    if (ctx->broken) return SPFC_E_DEVICE;
    return tune_ctx(ctx, dt, trial_steps, reinterpret_cast<char*>(scratch_dev));
}

int spfc_time_kernels(spfc_ctx* ctx, double dt, int reps, void* scratch_dev, size_t scratch_bytes) {
    const TraceRange trace_("spfc_time_kernels");
    if (!ctx || !scratch_dev || reps < 1) return SPFC_E_INVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return SPFC_E_INVAL;
    if (scratch_bytes < snapshot_bytes(ctx)) return SPFC_E_NOMEM;
    if (ctx->broken) return SPFC_E_DEVICE;
    return time_ctx(ctx, dt, reps, reinterpret_cast<char*>(scratch_dev));
}

int spfc_get_plan(spfc_ctx* ctx, int* plan8) {
    if (!ctx || !plan8) return SPFC_E_INVAL;
    get_plan(ctx, plan8);
    return SPFC_OK;
}

int spfc_destroy(spfc_ctx* ctx) {
    if (!ctx) return SPFC_E_INVAL;
    free_ctx(ctx);
    return SPFC_OK;
}

// ---------------------------------------------------------------- allocation-free run

// The workspace of spfc_run_noalloc: one array per device, part of the code object.
// Host code never takes its name as an address: the device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and kept.
static __device__ __align__(256) unsigned char scratch[SPFC_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

int scratch_of_current_device(char** ptr) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SPFC_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SPFC_E_DEVICE;
        if (reinterpret_cast<uintptr_t>(p) % kAlign) return SPFC_E_DEVICE;
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return SPFC_OK;
}

}  // namespace

int spfc_run_noalloc(const spfc_grid* grid, const spfc_params* params, const double* phi0_dev, double dt,
                     int64_t n, void* phi_out_dev, int dtype, spfc_energy_t* energy_out, void* hip_stream) {
    const TraceRange trace_("spfc_run_noalloc");
    if (!phi0_dev || !phi_out_dev || (dtype != SPFC_FP64 && dtype != SPFC_FP32)) return SPFC_E_INVAL;
    if (!(dt > 0.0) || !std::isfinite(dt) || n < 0) return SPFC_E_INVAL;
    int rc = validate(grid, params);
    if (rc) return rc;
    const size_t need = class_bytes(*grid, *params, 1);
    if (need > SPFC_NOALLOC_BYTES) return SPFC_E_NOMEM;
    char* ws = nullptr;
    if ((rc = scratch_of_current_device(&ws))) return rc;
    // spfc_init on the array (it clears the scalar blocks and the history; every field
    // region is written before it is read)
    spfc_ctx* ctx = nullptr;
    if ((rc = spfc_init(grid, params, phi0_dev, ws, SPFC_NOALLOC_BYTES, hip_stream, &ctx))) return rc;
    rc = ctx_step(ctx, dt, n);
    if (!rc) rc = ctx_get_phi(ctx, 0, phi_out_dev, dtype);
    if (!rc) {
        spfc_energy_t e{};
        rc = ctx_energy(ctx, 0, &e);
        if ((rc == SPFC_OK || rc == SPFC_E_NONFINITE) && energy_out) *energy_out = e;
    }
    if ((rc == SPFC_OK || rc == SPFC_E_NONFINITE) && hipStreamSynchronize(ctx->stream) != hipSuccess)
        rc = SPFC_E_DEVICE;
    free_ctx(ctx);
    return rc;
}

// ---------------------------------------------------------------- batches

int spfc_batch_workspace_bytes(int count, const spfc_grid* grids, const spfc_params* params, size_t* bytes) {
    if (!bytes) return SPFC_E_INVAL;
    const int rc = validate_batch(count, grids, params);
    if (rc) return rc;
    *bytes = batch_bytes(group_members(count, grids, params), grids, params);
    return SPFC_OK;
}

int spfc_batch_init(int count, const spfc_grid* grids, const spfc_params* params, const double* const* phi0_dev,
                    void* workspace_dev, size_t workspace_bytes, void* hip_stream, spfc_batch** out) {
    const TraceRange trace_("spfc_batch_init");
    if (!out || !phi0_dev || !workspace_dev) return SPFC_E_INVAL;
    int rc = validate_batch(count, grids, params);
    if (rc) return rc;
    if (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign) return SPFC_E_INVAL;
    const auto classes = group_members(count, grids, params);
    if (workspace_bytes < batch_bytes(classes, grids, params)) return SPFC_E_NOMEM;
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    for (int i = 0; i < count; ++i) {
        if (!phi0_dev[i]) return SPFC_E_INVAL;
        const Sizes s = sizes_of(grids[i], params[i].precision);
        if ((rc = check_finite_field(phi0_dev[i], (size_t)s.nx * s.ny * s.nz, stream))) return rc;
    }
    spfc_batch* b = new (std::nothrow) spfc_batch();
    if (!b) return SPFC_E_NOMEM;
    b->where.assign(count, {0, 0});
    for (int i = 0; i < count; ++i) {
        const Sizes s = sizes_of(grids[i], params[i].precision);
        b->npts.push_back((size_t)s.nx * s.ny * s.nz);
    }
    char* ws = reinterpret_cast<char*>(workspace_dev);
    for (size_t c = 0; c < classes.size(); ++c) {
        const auto& idx = classes[c];
        const int M = (int)idx.size();
        spfc_ctx* ctx = nullptr;
        rc = make_ctx(grids, params, idx.data(), M, phi0_dev, ws, stream, &ctx);
        if (rc) {
            for (auto* x : b->cls) free_ctx(x);
            delete b;
            return rc;
        }
        ws += class_bytes(grids[idx[0]], params[idx[0]], M);
        for (int k = 0; k < M; ++k) b->where[idx[k]] = {(int)c, k};
        b->cls.push_back(ctx);
        b->members.push_back(idx);
    }
    b->stream = stream;
    const char* serial = std::getenv("SPFC_BATCH_SERIAL");   // 1: classes one after another (for A/B timing)
    if (b->cls.size() > 1 && !(serial && serial[0] == '1')) {
        bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
        for (size_t c = 0; ok && c < b->cls.size(); ++c) {
            hipStream_t s = nullptr;
            hipEvent_t e = nullptr;
            ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
            if (ok) b->cstream.push_back(s);
            ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
            if (ok) b->join.push_back(e);
        }
        if (!ok) {
            spfc_batch_destroy(b);
            return SPFC_E_DEVICE;
        }
    }
    *out = b;
    return SPFC_OK;
}

int spfc_batch_set_graph(spfc_batch* b, int enable) {
    if (!b) return SPFC_E_INVAL;
    for (auto* c : b->cls) spfc_set_graph(c, enable);
    b->use_graph = enable != 0 && b->stream != nullptr;
    if (!b->use_graph) drop_batch_graphs(b);
    return SPFC_OK;
}

int spfc_batch_step(spfc_batch* b, double dt, int64_t n) {
    const TraceRange trace_("spfc_batch_step");
    if (!b) return SPFC_E_INVAL;
    if (!(dt > 0.0) || !std::isfinite(dt) || n < 0) return SPFC_E_INVAL;
    if (b->cstream.empty() || n == 0) {
        for (auto* c : b->cls) {
            const int rc = ctx_step(c, dt, n);
            if (rc) return rc;
        }
        return SPFC_OK;
    }
    // fork: every class stream waits for what the caller queued before this call
    int rc = batch_fork(b);
    for (size_t c = 0; c < b->cls.size(); ++c) b->cls[c]->stream = b->cstream[c];
    if (rc == SPFC_OK) {
        if (b->use_graph) {
            rc = batch_steps_graph(b, dt, n);
        } else {
            for (size_t c = 0; c < b->cls.size() && rc == SPFC_OK; ++c) rc = ctx_step(b->cls[c], dt, n);
        }
    }
    // join: the caller's stream waits for every class (also after an error, so that no
    // class work is left behind the caller's back)
    const int rj = batch_join(b);
    if (!rc) rc = rj;
    for (size_t c = 0; c < b->cls.size(); ++c) b->cls[c]->stream = b->stream;
    return rc;
}

int spfc_batch_step_count(spfc_batch* b, int64_t* n) {
    if (!b || !n) return SPFC_E_INVAL;
    *n = b->cls[0]->step;
    return SPFC_OK;
}

int spfc_batch_status(spfc_batch* b, int member, uint32_t* flags) {
    if (!member_ok(b, member) || !flags) return SPFC_E_INVAL;
    return ctx_status(b->cls[b->where[member].first], b->where[member].second, flags);
}

int spfc_batch_mass(spfc_batch* b, int member, double* mean) {
    if (!member_ok(b, member) || !mean) return SPFC_E_INVAL;
    return ctx_mass(b->cls[b->where[member].first], b->where[member].second, mean);
}

int spfc_batch_energy(spfc_batch* b, int member, spfc_energy_t* out) {
    if (!member_ok(b, member) || !out) return SPFC_E_INVAL;
    return ctx_energy(b->cls[b->where[member].first], b->where[member].second, out);
}

int spfc_batch_history(spfc_batch* b, int member, int64_t first, int64_t count, spfc_record* out) {
    if (!member_ok(b, member) || (!out && count > 0) || first < 0 || count < 0) return SPFC_E_INVAL;
    return ctx_history(b->cls[b->where[member].first], b->where[member].second, first, count, out);
}

int spfc_batch_get_phi(spfc_batch* b, int member, void* out_dev, int dtype) {
    if (!member_ok(b, member) || !out_dev || (dtype != SPFC_FP64 && dtype != SPFC_FP32)) return SPFC_E_INVAL;
    return ctx_get_phi(b->cls[b->where[member].first], b->where[member].second, out_dev, dtype);
}

int spfc_batch_profile(spfc_batch* b, int enable) {
    if (!b) return SPFC_E_INVAL;
    for (auto* c : b->cls) {
        const int rc = spfc_profile(c, enable);
        if (rc) return rc;
    }
    return SPFC_OK;
}

int spfc_batch_kernel_times(spfc_batch* b, int cap, const char** names, double* avg_ms, int64_t* launches,
                            double* bytes_per_launch, int* count) {
    if (!b || !count) return SPFC_E_INVAL;
    double ms[R_COUNT] = {0}, by[R_COUNT] = {0};
    int64_t nl[R_COUNT] = {0};
    for (auto* ctx : b->cls) {
        const int rc = drain_events(ctx);
        if (rc) return rc;
        const double F = (double)ctx->lay.F * ctx->M;
        const int d = ctx->sz.dim;
        const double bytes[R_COUNT] = {6.0 * F, 5.0 * F, 2.0 * d * F, 5.0 * F, 5.0 * F, 0.0};
        for (int i = 0; i < R_COUNT; ++i) {
            if (ctx->role_n[i] == 0) continue;
            ms[i] += ctx->role_ms[i] / (double)ctx->role_n[i];
            by[i] += bytes[i];
            nl[i] = std::max(nl[i], ctx->role_n[i]);
        }
    }
    int k = 0;
    for (int i = 0; i < R_COUNT; ++i) {
        if (nl[i] == 0) continue;
        if (k < cap) {
            if (names) names[k] = kRoleNames[i];
            if (avg_ms) avg_ms[k] = ms[i];
            if (launches) launches[k] = nl[i];
            if (bytes_per_launch) bytes_per_launch[k] = by[i];
        }
        ++k;
    }
    *count = k;
    return SPFC_OK;
}

int spfc_batch_tune_bytes(spfc_batch* b, size_t* bytes) {
    if (!b || !bytes) return SPFC_E_INVAL;
    size_t m = 0;
    for (auto* c : b->cls) m = std::max(m, snapshot_bytes(c));
    *bytes = m;
    return SPFC_OK;
}

int spfc_batch_tune(spfc_batch* b, double dt, int64_t trial_steps, void* scratch_dev, size_t scratch_bytes) {
    const TraceRange trace_("spfc_batch_tune");
    if (!b || !scratch_dev) return SPFC_E_INVAL;
    if (!(dt > 0.0) || !std::isfinite(dt) || trial_steps < 1) return SPFC_E_INVAL;
    for (auto* c : b->cls) {
        const int rc = spfc_tune(c, dt, trial_steps, scratch_dev, scratch_bytes);
        if (rc) return rc;
    }
    return SPFC_OK;
}

int spfc_batch_time_kernels(spfc_batch* b, double dt, int reps, void* scratch_dev, size_t scratch_bytes) {
    const TraceRange trace_("spfc_batch_time_kernels");
    if (!b) return SPFC_E_INVAL;
    for (auto* c : b->cls) {
        const int rc = spfc_time_kernels(c, dt, reps, scratch_dev, scratch_bytes);
        if (rc) return rc;
    }
    return SPFC_OK;
}

int spfc_batch_get_plan(spfc_batch* b, int member, int* plan8) {
    if (!member_ok(b, member) || !plan8) return SPFC_E_INVAL;
    get_plan(b->cls[b->where[member].first], plan8);
    return SPFC_OK;
}

int spfc_batch_reset(spfc_batch* b, const double* const* phi_dev, const double* r_shift) {
    const TraceRange trace_("spfc_batch_reset");
    if (!b || !phi_dev) return SPFC_E_INVAL;
    for (size_t i = 0; i < b->npts.size(); ++i) {
        if (!phi_dev[i]) return SPFC_E_INVAL;
        if (r_shift && !std::isfinite(r_shift[i])) return SPFC_E_INVAL;
    }
    int worst = SPFC_OK;
    for (size_t c = 0; c < b->cls.size(); ++c) {
        spfc_ctx* ctx = b->cls[c];
        const int rc = reset_ctx(ctx, b->members[c].data(), phi_dev);
        if (rc) return rc;
        if (r_shift) {
            // the restart pass left r = sqrt(E_1(phi)) in both levels of the pair
            std::vector<DevScalars> sc(ctx->M);
            CK(hipMemcpyAsync(sc.data(), ctx->sc(0), ctx->M * sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->stream));
            CK(hipStreamSynchronize(ctx->stream));
            for (int m = 0; m < ctx->M; ++m) {
                const double r = sc[m].r_n + r_shift[b->members[c][m]];
                if (r > 0.0) {
                    sc[m].r_n = sc[m].r_nm1 = r;
                } else {
                    worst = SPFC_E_INVAL;
                }
            }
            CK(hipMemcpyAsync(ctx->sc(0), sc.data(), ctx->M * sizeof(DevScalars), hipMemcpyHostToDevice, ctx->stream));
            CK(hipStreamSynchronize(ctx->stream));
        }
    }
    return worst;
}

int spfc_batch_get_phi_all(spfc_batch* b, void* const* out_dev, int dtype) {
    const TraceRange trace_("spfc_batch_get_phi_all");
    if (!b || !out_dev || (dtype != SPFC_FP64 && dtype != SPFC_FP32)) return SPFC_E_INVAL;
    for (size_t i = 0; i < b->npts.size(); ++i)
        if (!out_dev[i]) return SPFC_E_INVAL;
    for (size_t c = 0; c < b->cls.size(); ++c) {
        spfc_ctx* ctx = b->cls[c];
        if (ctx->broken) return SPFC_E_DEVICE;
        std::vector<void*> out(ctx->M);
        for (int m = 0; m < ctx->M; ++m) out[m] = out_dev[b->members[c][m]];
        const int rc = with_pipe(ctx, [&](auto& p) { return p.inverse_real(0, ctx->M, out.data(), dtype == SPFC_FP32); });
        if (rc) return rc;
    }
    return SPFC_OK;
}

int spfc_batch_energies(spfc_batch* b, spfc_energy_t* out) {
    const TraceRange trace_("spfc_batch_energies");
    if (!b || !out) return SPFC_E_INVAL;
    int worst = SPFC_OK;
    for (size_t c = 0; c < b->cls.size(); ++c) {
        spfc_ctx* ctx = b->cls[c];
        if (ctx->broken) return SPFC_E_DEVICE;
        int rc = with_pipe(ctx, [&](auto& p) {
            return p.e1_pass(ctx->slot(ctx->slotX), ctx->slot(ctx->slotY), FIN_QUERY);
        });
        if (rc) return rc;
        std::vector<DevScalars> sc(ctx->M);
        CK(hipMemcpyAsync(sc.data(), ctx->sc(0), ctx->M * sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        for (int m = 0; m < ctx->M; ++m) {
            const Geo& g = ctx->geos[m];
            const DevScalars& d = sc[m];
            spfc_energy_t& e = out[b->members[c][m]];
            const double rn = d.r_n, rm = d.r_nm1;
            e.modified_energy = 0.25 * (d.q_norm[0] + d.q_norm[1]) + 0.5 * (rn * rn + (2 * rn - rm) * (2 * rn - rm)) +
                                0.25 * g.stab * ctx->dt_prev * d.q_norm[4];
            e.E1 = d.q_E1;
            e.energy = d.q_E1 - g.e1_const + 0.5 * g.a * d.q_norm[2] + 0.5 * d.q_norm[3];
            e.sav_energy = 0.5 * g.a * d.q_norm[2] + 0.5 * d.q_norm[3] + rn * rn;
            e.r = rn;
            e.mean = d.mean;
            e.step = ctx->step;
            if (d.flags & SPFC_FLAG_NONFINITE) worst = SPFC_E_NONFINITE;
        }
    }
    return worst;
}

int spfc_batch_destroy(spfc_batch* b) {
    if (!b) return SPFC_E_INVAL;
    drop_batch_graphs(b);
    for (auto* c : b->cls) free_ctx(c);
    for (auto s : b->cstream) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (auto e : b->join) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
    return SPFC_OK;
}

}  // extern "C"
