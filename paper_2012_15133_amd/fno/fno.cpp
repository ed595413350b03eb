// Host driver and C ABI of the FNO surrogate (include/spfc_fno.h): workspace carving,
// forward pass, backward pass (reverse of the forward, one layer at a time) and Adam.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <new>
#include <vector>

#include "fno_kernels.hpp"
#include "trace.hpp"
#include "spfc_fno.h"

using namespace fno;

namespace {

constexpr int OK = 0, E_INVAL = 1, E_NOMEM = 2, E_DEVICE = 3;
constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t prm, wpk, tw, bx, bxt, ta, ts, xp, zz, v, u, w, ga, gb, vh, uh, gvh, out_raw, pred, gpred, lpart, gpart, partials,
        grad, m, vv, total;
    size_t field_bf, field_f, spec;   // bytes of one activation (bf16), one f32 field set, one spectrum set
};

bool shape_ok(const spfc_fno_shape* s) {
    return s && (s->n == 64 || s->n == 128 || s->n == 256) && s->max_batch >= 1 && s->max_batch <= 128 &&
           (s->train == 0 || s->train == 1);
}

Layout layout_of(const spfc_fno_shape& s) {
    Layout L{};
    const size_t npts = (size_t)s.n * s.n, planes = (size_t)s.max_batch * C;
    const size_t nwg = npts / TPB;
    L.field_bf = planes * npts * sizeof(uint16_t);
    L.field_f = planes * npts * sizeof(float);
    L.spec = (size_t)NMODE * planes * sizeof(float2);
    const bool tr = s.train != 0;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes);
        return at;
    };
    L.prm = take(P_TOTAL * sizeof(float));
    L.wpk = take((size_t)LAYERS * NMODE * 64 * 64 * sizeof(uint16_t));
    L.tw = take((size_t)s.n * sizeof(float2));
    L.bx = take(2 * (size_t)s.n * 2 * MX * sizeof(uint16_t));
    L.bxt = take(2 * (size_t)s.n * 2 * MX * sizeof(uint16_t));
    L.ta = take(4 * (size_t)s.n * 2 * MY * sizeof(uint16_t));
    L.ts = take(4 * (size_t)s.n * 2 * MY * sizeof(uint16_t));
    L.xp = take(planes * s.n * 2 * MX * sizeof(float));
    L.zz = take(planes * s.n * 2 * MX * sizeof(float));
    L.v = take((tr ? LAYERS + 1 : 2) * align_up(L.field_bf));
    L.u = take(tr ? LAYERS * align_up(L.field_bf) : 0);
    L.w = take(L.field_f);
    L.ga = take(tr ? L.field_f : 0);
    L.gb = take(tr ? L.field_f : 0);
    L.vh = take((tr ? LAYERS : 1) * align_up(L.spec));
    L.uh = take(L.spec);
    L.gvh = take(tr ? L.spec : 0);
    L.out_raw = take((size_t)s.max_batch * npts * sizeof(float));
    L.pred = take(tr ? (size_t)s.max_batch * npts * sizeof(float) : 0);
    L.gpred = take(tr ? (size_t)s.max_batch * npts * sizeof(float) : 0);
    L.lpart = take((size_t)s.max_batch * nwg * sizeof(float));
    L.gpart = take((size_t)s.max_batch * nwg * sizeof(float));
    L.partials = take(tr ? (size_t)GRED64 * PART_MAX * sizeof(float) : 0);
    L.grad = take(tr ? P_TOTAL * sizeof(float) : 0);
    L.m = take(tr ? P_TOTAL * sizeof(float) : 0);
    L.vv = take(tr ? P_TOTAL * sizeof(float) : 0);
    L.total = o;
    return L;
}

}  // namespace

// kernel roles of the forward pass (per-kernel timing)
enum { FR_LIFT = 0, FR_COL_ANAL, FR_MIX, FR_COL_SYNTH, FR_LAYER, FR_LAST, FR_FILTER_ANAL, FR_FILTER_SYNTH, FR_FINISH,
       FR_COUNT };
const char* const kFnoRoles[FR_COUNT] = {"lift_row", "col_anal", "mix", "col_synth", "layer_row", "last_row",
                                         "filter_anal", "filter_synth", "finish"};

struct spfc_fno {
    spfc_fno_shape shape;
    Layout lay;
    char* ws;
    hipStream_t stream;
    int64_t adam_t;
    bool broken;
    // per-kernel timing of a forward pass (reps > 0 while spfc_fno_time_forward runs)
    int reps = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double role_ms[FR_COUNT] = {}, role_bytes[FR_COUNT] = {};
    int role_n[FR_COUNT] = {};

    template <typename T>
    T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    float* prm() const { return at<float>(lay.prm); }
    uint16_t* wpk(int l) const { return at<uint16_t>(lay.wpk) + (size_t)l * NMODE * 64 * 64; }
    const float2* tw() const { return at<float2>(lay.tw); }
    uint16_t* v(int l) const {
        const int slot = shape.train ? l : (l & 1);
        return reinterpret_cast<uint16_t*>(ws + lay.v + slot * align_up(lay.field_bf));
    }
    uint16_t* u(int l) const {
        return shape.train ? reinterpret_cast<uint16_t*>(ws + lay.u + l * align_up(lay.field_bf)) : nullptr;
    }
    float* w() const { return at<float>(lay.w); }
    float2* vh(int l) const {
        return reinterpret_cast<float2*>(ws + lay.vh + (shape.train ? l : 0) * align_up(lay.spec));
    }
    float2* uh() const { return at<float2>(lay.uh); }
    float2* gvh() const { return at<float2>(lay.gvh); }
    float* xp() const { return at<float>(lay.xp); }
    float* zz() const { return at<float>(lay.zz); }
    const uint16_t* bx() const { return at<uint16_t>(lay.bx); }
    const uint16_t* bxt() const { return at<uint16_t>(lay.bxt); }
    const uint16_t* ta() const { return at<uint16_t>(lay.ta); }
    const uint16_t* ts() const { return at<uint16_t>(lay.ts); }
};

namespace {

#define CK(x)                    \
    do {                         \
        hipError_t e_ = (x);     \
        if (e_ != hipSuccess) {  \
            f->broken = true;    \
            return E_DEVICE;     \
        }                        \
    } while (0)

// One launch of a forward-pass kernel; while timing, `reps` back-to-back launches between
// two events on the stream (every launch of the pass is idempotent).
template <class L>
int run_role(spfc_fno* f, int role, double bytes, L&& launch) {
    if (f->reps <= 0) {
        CK(launch());
        return OK;
    }
    CK(hipEventRecord(f->ev0, f->stream));
    for (int r = 0; r < f->reps; ++r) CK(launch());
    CK(hipEventRecord(f->ev1, f->stream));
    CK(hipEventSynchronize(f->ev1));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, f->ev0, f->ev1));
    f->role_ms[role] += (double)ms / f->reps;
    f->role_bytes[role] = bytes;
    f->role_n[role] += 1;
    return OK;
}

int pack_all(spfc_fno* f) {
    for (int l = 0; l < LAYERS; ++l)
        CK(launch_pack_weights(f->prm() + p_wr(l), f->prm() + p_wi(l), f->wpk(l), f->stream));
    return OK;
}

// Forward pass for `batch` samples; with a target also the loss pieces (gpred etc.).
int forward(spfc_fno* f, int batch, const float* phi, const float* eps, const float* target, float* pred) {
    const int n = f->shape.n, planes = batch * C;
    const float inv = 1.0f / ((float)n * (float)n);
    hipStream_t st = f->stream;
    const bool tr = f->shape.train != 0 && target;
    int rc;
    // algorithmic bytes of each role (reads + writes): activations bf16, X' and Z FP32
    // [32][n][planes], spectra float2 [512][planes]
    const double N = n, P = planes, B = batch;
    const double act = P * N * N * 2, xz = 32.0 * N * P * 4, spec = (double)NMODE * P * 8;
    const double xz1 = 32.0 * N * B * 4, spec1 = (double)NMODE * B * 8, fld = B * N * N * 4;
    // rows: lifting + x-analysis; per layer: y-analysis, mixing, y-synthesis, then the row
    // kernel (x-synthesis, pointwise layer, activation, next x-analysis; the last layer's
    // row kernel also projects and takes the x-analysis of the output)
    RowIn in{};
    in.phi = phi;
    in.eps = eps;
    in.prm = f->prm();
    in.bx = f->bx();
    in.bxt = f->bxt();
    in.tw = f->tw();
    in.vout = f->v(0);
    in.xout = f->xp();
    if ((rc = run_role(f, FR_LIFT, fld + act + xz, [&] { return launch_row(n, batch, RK_LIFT, in, st); }))) return rc;
    // the output's x-analysis goes to out_raw's space (free during the forward pass)
    float* xo = f->at<float>(f->lay.out_raw);
    for (int l = 0; l < LAYERS; ++l) {
        const bool last = l == LAYERS - 1;
        if ((rc = run_role(f, FR_COL_ANAL, xz + spec,
                           [&] { return launch_col_anal(n, planes, f->xp(), inv, f->vh(l), f->ta(), st); })))
            return rc;
        if ((rc = run_role(f, FR_MIX, 2 * spec + (double)NMODE * 64 * 64 * 2, [&] {
                 return launch_mix(MIX_FWD, batch, f->vh(l), nullptr, f->wpk(l), f->uh(), nullptr, nullptr, st);
             })))
            return rc;
        if ((rc = run_role(f, FR_COL_SYNTH, spec + xz,
                           [&] { return launch_col_synth(n, planes, f->uh(), 1.0f, 2.0f, false, f->zz(), f->ts(), st); })))
            return rc;
        in.layer = l;
        in.Z = f->zz();
        in.v = f->v(l);
        in.vout = (!last || tr) ? f->v(l + 1) : nullptr;
        in.uout = (tr && !last) ? f->u(l) : nullptr;
        in.xout = last ? xo : f->xp();
        const double bytes = last ? act + xz + xz1 + (in.vout ? act : 0.0)
                                  : 2 * act + 2 * xz + (in.uout ? act : 0.0);
        if ((rc = run_role(f, last ? FR_LAST : FR_LAYER, bytes,
                           [&] { return launch_row(n, batch, last ? RK_LAST : RK_LAYER, in, st); })))
            return rc;
    }
    // the increment restricted to the retained modes, without its mean (the k = 0 mode
    // dropped), added to phi
    if ((rc = run_role(f, FR_FILTER_ANAL, xz1 + spec1,
                       [&] { return launch_col_anal(n, batch, xo, inv, f->uh(), f->ta(), st); })))
        return rc;
    if ((rc = run_role(f, FR_FILTER_SYNTH, spec1 + xz1,
                       [&] { return launch_col_synth(n, batch, f->uh(), 1.0f, 2.0f, true, f->zz(), f->ts(), st); })))
        return rc;
    return run_role(f, FR_FINISH, 2 * fld + xz1 + (target ? 2 * fld : 0.0), [&] {
        return launch_finish(n, batch, phi, f->zz(), f->tw(), target, pred, tr ? f->at<float>(f->lay.gpred) : nullptr,
                             f->at<float>(f->lay.lpart), f->at<float>(f->lay.gpart), st);
    });
}

// Loss and gradient into the internal gradient buffer and loss_dev.
int backward(spfc_fno* f, int batch, const float* phi, const float* eps, const float* target, float* loss_dev) {
    const int n = f->shape.n, planes = batch * C;
    const int nwg = n * n / TPB;
    const float inv = 1.0f / ((float)n * (float)n);
    hipStream_t st = f->stream;
    int rc;
    if ((rc = forward(f, batch, phi, eps, target, f->at<float>(f->lay.pred)))) return rc;
    float* grad = f->at<float>(f->lay.grad);
    float* partials = f->at<float>(f->lay.partials);
    CK(launch_reduce(f->at<float>(f->lay.lpart), batch * nwg, 1, inv / (float)batch, loss_dev, st));
    float* ga = f->at<float>(f->lay.ga);
    float* gb = f->at<float>(f->lay.gb);
    // adjoints of the mean restoration and of the filter (synth o anal)^T = anal^T synth^T
    float* gcen = f->at<float>(f->lay.out_raw);
    float* gout = f->at<float>(f->lay.pred);
    CK(launch_center(n, batch, f->at<float>(f->lay.gpred), f->at<float>(f->lay.gpart), gcen, st));
    CK(launch_analysis_f32(n, batch, gcen, 1.0f, 2.0f, f->uh(), f->tw(), st));
    CK(launch_synthesis(n, batch, f->uh(), inv, inv, gout, 0, f->tw(), st));
    CK(launch_project_bwd(n, batch, f->v(LAYERS), f->prm(), gout, ga, partials, st));
    CK(launch_reduce(partials, GRED64, PART_PROJ, 1.0f, grad + P_Q1, st));
    for (int l = LAYERS - 1; l >= 0; --l) {
        float* gu = f->w();
        CK(launch_pointwise_bwd(n, batch, l < LAYERS - 1, ga, f->u(l), f->v(l), f->prm() + p_pw(l), gu, gb, partials,
                                st));
        CK(launch_reduce(partials, GRED64, PART_PW, 1.0f, grad + p_pw(l), st));
        // adjoint of the synthesis: analysis with the synthesis weights and no 1/N^2
        CK(launch_analysis_f32(n, planes, gu, 1.0f, 2.0f, f->uh(), f->tw(), st));
        CK(launch_mix(MIX_BWD_WEIGHT, batch, f->vh(l), f->uh(), nullptr, nullptr, grad + p_wr(l), grad + p_wi(l),
                      st));
        CK(launch_mix(MIX_BWD_DATA, batch, f->uh(), nullptr, f->wpk(l), f->gvh(), nullptr, nullptr, st));
        // adjoint of the analysis: synthesis with weight 1/N^2 on every mode, added to gv
        CK(launch_synthesis(n, planes, f->gvh(), inv, inv, gb, 1, f->tw(), st));
        std::swap(ga, gb);
    }
    CK(launch_lift_bwd(n, batch, ga, phi, eps, partials, st));
    CK(launch_reduce(partials, GRED, PART_LIFT, 1.0f, grad + P_LW, st));
    return OK;
}

int check_call(spfc_fno* f, int batch) {
    if (!f) return E_INVAL;
    if (f->broken) return E_DEVICE;
    if (batch < 1 || batch > f->shape.max_batch) return E_INVAL;
    return OK;
}

}  // namespace

extern "C" {

int spfc_fno_param_count(int64_t* count) {
    if (!count) return E_INVAL;
    *count = P_TOTAL;
    return OK;
}

int spfc_fno_workspace_bytes(const spfc_fno_shape* shape, size_t* bytes) {
    if (!bytes || !shape_ok(shape)) return E_INVAL;
    *bytes = layout_of(*shape).total;
    return OK;
}

int spfc_fno_init(const spfc_fno_shape* shape, const float* params_dev, void* workspace_dev, size_t workspace_bytes,
                  void* hip_stream, spfc_fno** out) {
    const spfc::TraceRange trace_("spfc_fno_init");
    if (!out || !params_dev || !workspace_dev || !shape_ok(shape)) return E_INVAL;
    if (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign) return E_INVAL;
    const Layout lay = layout_of(*shape);
    if (workspace_bytes < lay.total) return E_NOMEM;
    spfc_fno* f = new (std::nothrow) spfc_fno();
    if (!f) return E_NOMEM;
    f->shape = *shape;
    f->lay = lay;
    f->ws = reinterpret_cast<char*>(workspace_dev);
    f->stream = reinterpret_cast<hipStream_t>(hip_stream);
    f->adam_t = 0;
    f->broken = false;
    std::vector<float2> tw(shape->n);
    for (int j = 0; j < shape->n; ++j) {
        const double a = 2.0 * 3.14159265358979323846 * j / shape->n;
        tw[j] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    auto fail = [&](int code) {
        delete f;
        return code;
    };
    if (hipMemcpyAsync(f->prm(), params_dev, P_TOTAL * sizeof(float), hipMemcpyDeviceToDevice, f->stream) !=
        hipSuccess)
        return fail(E_DEVICE);
    if (hipMemcpyAsync(f->ws + lay.tw, tw.data(), shape->n * sizeof(float2), hipMemcpyHostToDevice, f->stream) !=
        hipSuccess)
        return fail(E_DEVICE);
    if (shape->train) {
        if (hipMemsetAsync(f->ws + lay.m, 0, lay.vv - lay.m + align_up(P_TOTAL * sizeof(float)), f->stream) !=
            hipSuccess)
            return fail(E_DEVICE);
    }
    if (pack_all(f)) return fail(E_DEVICE);
    if (launch_basis(shape->n, f->at<uint16_t>(lay.bx), f->at<uint16_t>(lay.bxt), f->stream) != hipSuccess ||
        launch_trig(shape->n, f->at<uint16_t>(lay.ta), f->at<uint16_t>(lay.ts), f->stream) != hipSuccess)
        return fail(E_DEVICE);
    if (hipStreamSynchronize(f->stream) != hipSuccess) return fail(E_DEVICE);
    *out = f;
    return OK;
}

int spfc_fno_forward(spfc_fno* f, int batch, const float* phi_dev, const float* eps_dev, float* out_dev) {
    const spfc::TraceRange trace_("spfc_fno_forward");
    int rc = check_call(f, batch);
    if (rc) return rc;
    if (!phi_dev || !eps_dev || !out_dev) return E_INVAL;
    return forward(f, batch, phi_dev, eps_dev, nullptr, out_dev);
}

int spfc_fno_time_forward(spfc_fno* f, int batch, const float* phi_dev, const float* eps_dev, float* out_dev, int reps,
                          int cap, const char** names, double* avg_ms, double* bytes, int* launches, int* count) {
    const spfc::TraceRange trace_("spfc_fno_time_forward");
    int rc = check_call(f, batch);
    if (rc) return rc;
    if (!phi_dev || !eps_dev || !out_dev || (const float*)out_dev == phi_dev || reps < 1 || reps > 1000 || !count || cap < 0 ||
        (cap > 0 && (!names || !avg_ms || !bytes || !launches)))
        return E_INVAL;
    if (!f->ev0 && (hipEventCreate(&f->ev0) != hipSuccess || hipEventCreate(&f->ev1) != hipSuccess)) {
        f->broken = true;
        return E_DEVICE;
    }
    for (int i = 0; i < FR_COUNT; ++i) {
        f->role_ms[i] = f->role_bytes[i] = 0.0;
        f->role_n[i] = 0;
    }
    f->reps = reps;
    rc = forward(f, batch, phi_dev, eps_dev, nullptr, out_dev);
    f->reps = 0;
    if (rc) return rc;
    int k = 0;
    for (int i = 0; i < FR_COUNT; ++i) {
        if (f->role_n[i] == 0) continue;
        if (k < cap) {
            names[k] = kFnoRoles[i];
            avg_ms[k] = f->role_ms[i] / f->role_n[i];
            bytes[k] = f->role_bytes[i];
            launches[k] = f->role_n[i];
        }
        ++k;
    }
    *count = k;
    return OK;
}

int spfc_fno_grads(spfc_fno* f, int batch, const float* phi_dev, const float* eps_dev, const float* target_dev,
                   float* loss_dev, float* grad_dev) {
    const spfc::TraceRange trace_("spfc_fno_grads");
    int rc = check_call(f, batch);
    if (rc) return rc;
    if (!f->shape.train || !phi_dev || !eps_dev || !target_dev || !loss_dev || !grad_dev) return E_INVAL;
    if ((rc = backward(f, batch, phi_dev, eps_dev, target_dev, loss_dev))) return rc;
    CK(hipMemcpyAsync(grad_dev, f->ws + f->lay.grad, P_TOTAL * sizeof(float), hipMemcpyDeviceToDevice, f->stream));
    return OK;
}

int spfc_fno_train_step(spfc_fno* f, int batch, const float* phi_dev, const float* eps_dev, const float* target_dev,
                        float lr, float* loss_dev) {
    const spfc::TraceRange trace_("spfc_fno_train_step");
    int rc = check_call(f, batch);
    if (rc) return rc;
    if (!f->shape.train || !phi_dev || !eps_dev || !target_dev || !loss_dev || !(lr > 0.f) || !std::isfinite(lr))
        return E_INVAL;
    if ((rc = backward(f, batch, phi_dev, eps_dev, target_dev, loss_dev))) return rc;
    f->adam_t += 1;
    const float c1 = 1.0f - (float)std::pow(0.9, (double)f->adam_t);
    const float c2 = 1.0f - (float)std::pow(0.999, (double)f->adam_t);
    CK(launch_adam(P_TOTAL, f->prm(), f->at<float>(f->lay.grad), f->at<float>(f->lay.m), f->at<float>(f->lay.vv), lr,
                   c1, c2, f->stream));
    return pack_all(f);
}

int spfc_fno_get_params(spfc_fno* f, float* params_dev) {
    if (!f || !params_dev) return E_INVAL;
    if (f->broken) return E_DEVICE;
    CK(hipMemcpyAsync(params_dev, f->prm(), P_TOTAL * sizeof(float), hipMemcpyDeviceToDevice, f->stream));
    return OK;
}

int spfc_fno_destroy(spfc_fno* f) {
    if (!f) return E_INVAL;
    if (!f->broken) (void)hipStreamSynchronize(f->stream);
    if (f->ev0) (void)hipEventDestroy(f->ev0);
    if (f->ev1) (void)hipEventDestroy(f->ev1);
    delete f;
    return OK;
}

}  // extern "C"
