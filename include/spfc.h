/*
 * spfc.h - C ABI of the GPU time stepper for the square phase field crystal
 * (SPFC) equation with the second-order SAV-BDF2 scheme of
 * M. Wang, Q. Huang, C. Wang, arXiv 2012.15133.
 *
 * Problem (Section 1, eq. equation-SPFC): on a periodic box of side L_j,
 *     d_t phi = Delta mu,  mu = -c4 div(|grad phi|^2 grad phi) + a phi + 2 Delta phi + Delta^2 phi,
 * a = 1 - epsilon > 0 and c4 = 1 in the paper.  Space: Fourier pseudo-spectral
 * collocation on n_x x n_y (x n_z) points (Section 2.1).  Time: the SAV scheme
 * eq. scheme-SAV-1 solved as in Section 2.3 (two constant-coefficient Fourier
 * solves and one scalar equation per step).
 *
 * Conventions shared by every call:
 *  - Real grid functions are arrays x-fastest: index x + n_x*(y + n_y*z).
 *  - Derivatives of odd order drop the Nyquist mode, those of even order keep it
 *    (the paper assumes odd n; its experiments and this library use even n).
 *  - Every pointer argument whose name ends in _dev is device memory of the
 *    current HIP device; all others are host memory.
 *  - All calls return an int status (SPFC_OK or an SPFC_E_* code) and leave their
 *    outputs untouched on error.  No exception crosses this boundary.
 *  - One host thread at a time per context.
 *  - The library allocates no device memory: the caller passes a workspace
 *    that must stay alive and untouched until spfc_destroy.  (The one exception
 *    is the fixed array that serves spfc_run_noalloc, which comes with the
 *    library's code object.)
 */
#ifndef SPFC_H
#define SPFC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    SPFC_OK = 0,
    SPFC_E_INVAL = 1,      /* bad argument: null pointer, unsupported size, a <= 0, dt <= 0, NaN input ... */
    SPFC_E_NOMEM = 2,      /* workspace smaller than spfc_workspace_bytes() */
    SPFC_E_DEVICE = 3,     /* a HIP call failed; the context is unusable afterwards */
    SPFC_E_NONFINITE = 4,  /* a query found the sticky NONFINITE flag set */
    SPFC_E_STATE = 5       /* call out of order (e.g. history not held), or bad checkpoint size */
};

/* sticky flags reported by spfc_status */
enum {
    SPFC_FLAG_NONFINITE = 1u,       /* E_1, an inner product or xi was not finite */
    SPFC_FLAG_E1_BELOW_OMEGA = 2u,  /* E_1 < |Omega|, against eq. energy-SPFC-split-2-2 */
    SPFC_FLAG_P1_POSITIVE = 4u,     /* <N, A^-1 Delta N> > 0, against eq. solver-5 */
    SPFC_FLAG_ENERGY_RISE = 8u      /* modified energy rose by more than energy_tol (Theorem 3.1) */
};

/* start-up of the two-step scheme */
enum {
    SPFC_STARTUP_SAV1 = 0,   /* first step: first-order SAV (weights (1,1,0), phihat = phi^0) */
    SPFC_STARTUP_GHOST = 1,  /* phi^-1 = phi^0 - dt Delta_N mu^0 (eq. scheme-SAV-initial-1) */
    SPFC_STARTUP_COPY = 2    /* phi^-1 = phi^0, r^-1 = r^0 (the restart rule of Section 5.2) */
};

/* storage and transform precision (inner products, energies, r and xi are FP64 in both) */
enum { SPFC_FP64 = 0, SPFC_FP32 = 1 };

typedef struct spfc_ctx spfc_ctx;
typedef struct spfc_batch spfc_batch;

/* Grid (Section 2.1).  dim = 2 or 3; n[j] points along axis j (x, y, z), each a
 * power of two in [8, 1024]; L[j] > 0 the box side.  Unused entries ignored. */
typedef struct {
    int dim;
    int n[3];
    double L[3];
} spfc_grid;

/* Model and run parameters.
 *  epsilon  : a = 1 - epsilon must be > 0 (Section 1).
 *  c4       : > 0, multiplies (1/4)|grad phi|^4 in the energy (paper: 1).  E_1 then carries
 *             the constant (1 + 1/c4)|Omega| (= 2|Omega| at c4 = 1, Section 2.2).
 *  startup  : SPFC_STARTUP_*.
 *  precision: SPFC_FP64 or SPFC_FP32.
 *  history  : capacity of the per-step record ring (>= 1).
 *  energy_tol: relative rise of the modified energy that sets SPFC_FLAG_ENERGY_RISE
 *             (<= 0 picks 1e-12 for FP64, 1e-6 for FP32).
 *  stab     : A >= 0.  A > 0 selects the stabilized scheme of the closing remarks of
 *             Section 5: the regularization -A dt Delta_N (phi^{n+1} - phi^n) is added to
 *             the chemical potential of every step (the step operator gains A dt^2 |k|^4,
 *             its right-hand side A dt^2 |k|^4 phi^n), and the modified energy gains
 *             (A dt / 4) <phi^n - phi^{n-1}, -Delta_N (phi^n - phi^{n-1})>, with which it
 *             is again non-increasing.  0 = the scheme eq. scheme-SAV-1.
 *  beta     : >= 0.  Adds (beta/4) phi^4 to the energy density, the quartic term of the
 *             standard PFC energy (Section 1, eq. energy-PFC), beside the 4-Laplacian term
 *             (0 = the SPFC energy of the paper).  Being convex and nonnegative it joins the
 *             nonlinear part: E_1 gains (beta/4)||phi||_4^4 (E_1 >= |Omega| still holds),
 *             N gains beta phi^3, E_N gains (beta/4)||phi||_4^4.  Any beta > 0 in a batch
 *             class runs the class on the kernels that carry phi to real space. */
typedef struct {
    double epsilon;
    double c4;
    int startup;
    int precision;
    int64_t history;
    double energy_tol;
    double stab;
    double beta;
} spfc_params;

/* Per-step record (index n = state phi^n).  energy is the modified energy
 * E(phi^n, phi^{n-1}, r^n, r^{n-1}) of Theorem 3.1 (eq. discrete energy; with the
 * stabilization term of spfc_params.stab when that is > 0), mean the
 * mean of phi^n, r = r^n.  xi = r^n / sqrt(E_1(phihat)), E1 = E_1(phihat) and
 * p1 = <N, A_N^-1 Delta_N N> belong to the step that produced phi^n (0 for n = 0). */
typedef struct {
    double energy;
    double mean;
    double r;
    double xi;
    double E1;
    double p1;
    double S;
    double reserved;
} spfc_record;

/* Energies of the current state phi^n (spfc_energy). */
typedef struct {
    double modified_energy;  /* E(phi^n, phi^{n-1}, r^n, r^{n-1}), Theorem 3.1 (+ stab term) */
    double energy;           /* E_N(phi^n), eq. energy-discrete-spectral (with c4) */
    double sav_energy;       /* a/2||phi||^2 + 1/2||Delta_N phi||^2 + r^2 (Section 5.2) */
    double r;                /* r^n */
    double E1;               /* E_{1,N}(phi^n) */
    double mean;             /* mean of phi^n */
    int64_t step;            /* n */
} spfc_energy_t;

/* Bytes of device workspace a context needs for this grid and parameters. */
int spfc_workspace_bytes(const spfc_grid* grid, const spfc_params* params, size_t* bytes);

/* Create a context.  phi0_dev: N_total doubles (x fastest), read during the call
 * only (the call synchronizes the stream before returning, so the caller may
 * free phi0_dev afterwards).  workspace_dev: at least spfc_workspace_bytes bytes,
 * 256-byte aligned, owned by the caller.  hip_stream: the hipStream_t every
 * later call enqueues on (0 = null stream).  Computes r^0 = sqrt(E_1(phi^0))
 * (after eq. scheme-SAV-initial-1).  Errors: SPFC_E_INVAL (bad grid/params,
 * null pointer, non-finite phi0, or a grid whose line transforms need more LDS
 * per workgroup than the device has, e.g. 3-D FP64 with n_x = 1024),
 * SPFC_E_NOMEM, SPFC_E_DEVICE. */
int spfc_init(const spfc_grid* grid, const spfc_params* params, const double* phi0_dev,
              void* workspace_dev, size_t workspace_bytes, void* hip_stream, spfc_ctx** out);

/* Advance n >= 0 steps of size dt > 0 (eq. scheme-SAV-1, solved as in Section 2.3).
 * The first step of a run uses the start-up mode.  A call with a dt different from
 * the previous one restarts the two-step scheme with phi^{-1} = phi^0 and
 * r = sqrt(E_1(phi^0)) at the current state (Section 5.2).  Asynchronous: only
 * kernel launches are enqueued.  Errors: SPFC_E_INVAL, SPFC_E_DEVICE. */
int spfc_step(spfc_ctx* ctx, double dt, int64_t n);

/* Forcing (the manufactured-solution test of Section 5.1, whose forcing the paper adds
 * without a formula): f(x, t) = sum_{i < terms} c_i(t) G_i(x), added to the phi equation
 * of every step at t^{n+1}, i.e. psi -> psi + dt f^{n+1} in the right-hand side of the
 * linear solve (eq. solver-3); the r equation (eq. solver-2) keeps a0 phi^{n+1} - psi.
 * spfc_forcing_bytes: device bytes the forcing needs (terms + 1 half spectra), 1 <= terms
 * <= SPFC_MAX_FORCING_TERMS.
 * spfc_set_forcing: g_dev[i] (device, n_z x n_y x n_x doubles, x fastest) is G_i; they
 * are transformed once into buf_dev (caller memory of spfc_forcing_bytes bytes, 256-byte
 * aligned, kept until the forcing is replaced or the context destroyed).  terms = 0
 * removes the forcing.  Synchronizes.
 * spfc_step_forced: as spfc_step, the s-th step of the call (s = 0 .. n - 1) with the
 * coefficients coef_dev[s * terms + i] = c_i(t^{n+1}) of its new time level (device
 * memory, read by the kernels as they run: keep it until the stream has passed them).
 * Direct launches (no graph replay).  Not offered with forcing (SPFC_E_INVAL): the ghost
 * start of a context that has not started (it would need f^0) and the stabilized scheme.
 * Errors: SPFC_E_INVAL (no forcing set, null or misaligned pointer, terms out of range,
 * buffer too small), SPFC_E_DEVICE. */
#define SPFC_MAX_FORCING_TERMS 16
int spfc_forcing_bytes(spfc_ctx* ctx, int terms, size_t* bytes);
int spfc_set_forcing(spfc_ctx* ctx, int terms, const double* const* g_dev, void* buf_dev, size_t bytes);
int spfc_step_forced(spfc_ctx* ctx, double dt, int64_t n, const double* coef_dev);

/* Mean of phi^n (synchronizes).  Theorem 2.1 keeps it at the mean of phi^0. */
int spfc_mass(spfc_ctx* ctx, double* mean);

/* Energies of the current state (synchronizes).  Returns SPFC_E_NONFINITE if the
 * NONFINITE flag is set (the struct is still filled). */
int spfc_energy(spfc_ctx* ctx, spfc_energy_t* out);

/* Copy records first .. first+count-1 to out (host).  SPFC_E_STATE if a record
 * is not held (not yet computed, or overwritten in the ring). Synchronizes. */
int spfc_history(spfc_ctx* ctx, int64_t first, int64_t count, spfc_record* out);

/* Number of the current step n (records 0..n exist). */
int spfc_step_count(spfc_ctx* ctx, int64_t* n);

/* Write phi^n in real space to out_dev (N_total values, x fastest), as doubles
 * (dtype SPFC_FP64) or floats (SPFC_FP32).  Asynchronous on the context stream. */
int spfc_get_phi(spfc_ctx* ctx, void* out_dev, int dtype);

/* Checkpoint: bytes needed, save into / load from caller device memory.  The state
 * is (phi^n, phi^{n-1}, r^n, r^{n-1}, n, dt of the last step, start-up status);
 * a run resumed from it continues bit for bit.  Synchronizes. */
int spfc_state_bytes(spfc_ctx* ctx, size_t* bytes);
int spfc_save_state(spfc_ctx* ctx, void* out_dev, size_t bytes);
int spfc_load_state(spfc_ctx* ctx, const void* in_dev, size_t bytes);

/* Sticky SPFC_FLAG_* bits (synchronizes). */
int spfc_status(spfc_ctx* ctx, uint32_t* flags);

/* Per-kernel timing of the step kernels, measured with HIP events on the context
 * stream.  spfc_profile(ctx, 1) starts recording (events around every launch of a
 * step kernel, which adds gaps between launches), 0 stops.  spfc_kernel_times
 * fills up to `cap` entries: name[i] (static string), average milliseconds per
 * launch, launches, and the algorithmic HBM bytes one launch must move.
 * Synchronizes. */
int spfc_profile(spfc_ctx* ctx, int enable);
int spfc_kernel_times(spfc_ctx* ctx, int cap, const char** names, double* avg_ms,
                      int64_t* launches, double* bytes_per_launch, int* count);

/* Graph replay (enable = 1): spfc_step then captures two steady BDF2 steps (the
 * launches of eq. scheme-SAV-1 with the weights 3/2, 2, -1/2 at one dt) into a HIP
 * graph on first use and replays it for each further pair of steps, which removes
 * the per-launch host cost.  Results are bit for bit those of direct launches.
 * Needs a non-null stream (on the null stream steps run directly); steps run
 * directly while profiling.  The graph is re-captured when dt changes.  Capture
 * uses hipStreamCaptureModeThreadLocal on the context stream, so nothing else may
 * be enqueued on that stream from another thread during spfc_step.  0 disables it
 * (default) and frees the graph. */
int spfc_set_graph(spfc_ctx* ctx, int enable);

/* Launch-plan tuner.  The step kernels run with a plan: for each of them the
 * values per thread (4, 8 or 16; the radix of the line transforms) and the
 * workgroup size.  spfc_tune times `trial_steps` steps of size dt > 0 for
 * candidate plans (a coordinate search over the kernels, 4/8/16 values per thread
 * x 128/256 threads) and keeps the fastest.  It starts every trial from a
 * snapshot of the run state (both states, scalars, history ring) that it keeps in
 * caller device memory scratch_dev of at least spfc_tune_bytes bytes, and
 * restores that state at the end, so the run continues from where it was; the
 * plan only changes the rounding of the transforms.  Synchronizes.  Errors:
 * SPFC_E_INVAL, SPFC_E_NOMEM (scratch too small), SPFC_E_DEVICE.
 * spfc_get_plan writes 8 ints: (values per thread, threads per workgroup) of the
 * gradient/inverse, real-space, forward and (3-D) middle-axis kernels, 0 where
 * unused. */
/* Kernel durations of a steady step of size dt > 0: from a snapshot of the run state
 * (in scratch_dev, spfc_tune_bytes bytes), one untimed step, then one step in which
 * each step kernel is launched `reps` >= 1 times back to back between two HIP
 * events on the context stream, so that the average is the kernel's own duration
 * rather than launch-to-launch time.  The repeats of the update kernel overwrite
 * the older state; the run state is restored from the snapshot at the end.  Read
 * the results with spfc_kernel_times.  Synchronizes.  Errors as spfc_tune. */
int spfc_time_kernels(spfc_ctx* ctx, double dt, int reps, void* scratch_dev, size_t scratch_bytes);
int spfc_tune_bytes(spfc_ctx* ctx, size_t* bytes);
int spfc_tune(spfc_ctx* ctx, double dt, int64_t trial_steps, void* scratch_dev, size_t scratch_bytes);
int spfc_get_plan(spfc_ctx* ctx, int* plan8);

/* ---------------------------------------------------------------- batches
 * A batch advances `count` independent runs ("members") together, e.g. a sweep
 * over epsilon, mean density or box size of Section 5.  Members of the same grid
 * sizes and precision form one class that shares every kernel launch (member m is
 * grid dimension y of each launch), so many small grids fill the GPU as one large
 * one would.  Members may differ in L and epsilon / c4; startup, history and
 * energy_tol must be equal for all members (else SPFC_E_INVAL).  Every member
 * follows exactly the arithmetic of a single run with its own grid and
 * parameters (same kernels, same reduction order), so its results equal those of
 * spfc_init + spfc_step on that member alone, bit for bit.
 * grids, params: `count` entries each (host).  phi0_dev: `count` device pointers
 * to the initial fields (N_total doubles of that member, x fastest), read during
 * the call only.  Workspace and stream as for spfc_init (one workspace for the
 * whole batch, from spfc_batch_workspace_bytes).  Member indices below are
 * positions in the arrays given to spfc_batch_init. */
int spfc_batch_workspace_bytes(int count, const spfc_grid* grids, const spfc_params* params,
                               size_t* bytes);
int spfc_batch_init(int count, const spfc_grid* grids, const spfc_params* params,
                    const double* const* phi0_dev, void* workspace_dev, size_t workspace_bytes,
                    void* hip_stream, spfc_batch** out);
/* Advance every member n steps of size dt (as spfc_step; asynchronous).  With several
 * size classes each class steps on a stream of its own that waits for the work queued
 * on the batch's stream before the call, and the batch's stream waits for every class
 * at the end, so the caller sees the steps ordered on the batch's stream. */
int spfc_batch_step(spfc_batch* b, double dt, int64_t n);
/* Graph replay (as spfc_set_graph).  With one size class the class's own graph is
 * replayed.  With several, one graph holds two steady steps of every class, each class
 * on a branch of its own (forked from the batch's stream and joined back into it), so
 * each further pair of steps of the whole batch is a single graph launch on the batch's
 * stream; it is captured again when dt, the plan or a class's state pair changes.
 * Results are bit for bit those of direct launches. */
int spfc_batch_set_graph(spfc_batch* b, int enable);
int spfc_batch_step_count(spfc_batch* b, int64_t* n);
/* Per-member queries, as their single-run counterparts; SPFC_E_INVAL for a member
 * index out of range.  spfc_batch_energy runs the query pass of the member's
 * whole class. */
int spfc_batch_status(spfc_batch* b, int member, uint32_t* flags);
int spfc_batch_mass(spfc_batch* b, int member, double* mean);
int spfc_batch_energy(spfc_batch* b, int member, spfc_energy_t* out);
int spfc_batch_history(spfc_batch* b, int member, int64_t first, int64_t count,
                       spfc_record* out);
int spfc_batch_get_phi(spfc_batch* b, int member, void* out_dev, int dtype);
/* Tune the plan of every class in turn (as spfc_tune; one scratch buffer of
 * spfc_batch_tune_bytes bytes serves all classes); read the plan of a member's class. */
int spfc_batch_tune_bytes(spfc_batch* b, size_t* bytes);
int spfc_batch_tune(spfc_batch* b, double dt, int64_t trial_steps, void* scratch_dev,
                    size_t scratch_bytes);
int spfc_batch_get_plan(spfc_batch* b, int member, int* plan8);
/* spfc_time_kernels for every class (scratch of spfc_batch_tune_bytes bytes); read the
 * results with spfc_batch_kernel_times. */
int spfc_batch_time_kernels(spfc_batch* b, double dt, int reps, void* scratch_dev,
                            size_t scratch_bytes);
/* Kernel timing as spfc_profile / spfc_kernel_times, summed over the classes: for
 * each step kernel, avg_ms is the sum over classes of its average launch time,
 * bytes_per_launch the algorithmic bytes of those launches together, launches the
 * count per class.  In spfc_batch_step the classes of a batch with several grid
 * sizes run on concurrent streams (forked from and joined to the batch's stream),
 * so these sums can exceed the wall time of a step; spfc_batch_time_kernels times
 * the classes one after another. */
int spfc_batch_profile(spfc_batch* b, int enable);
int spfc_batch_kernel_times(spfc_batch* b, int cap, const char** names, double* avg_ms,
                            int64_t* launches, double* bytes_per_launch, int* count);
/* Start every member's run again from new fields phi_dev[member] (as spfc_batch_init,
 * in the same workspace): step 0, the start-up mode on the next step, flags and
 * history cleared.  For a jump of a surrogate model or a restart from outside data.
 * The SAV variable of the new state (both levels of the pair) is sqrt(E_1(phi)) as at
 * init, plus r_shift[member] when r_shift (host, one finite value per member) is given:
 * a jump that keeps r - sqrt(E_1(phi)) of the state it leaves passes that difference.
 * A member whose shifted r would not be positive keeps sqrt(E_1(phi)) and the call
 * returns SPFC_E_INVAL after resetting every member.  The fields are not copied to the
 * host for a finiteness check (unlike init): a non-finite field sets the member's
 * NONFINITE flag in the E_1 pass of the restart.  Synchronizes.
 * Errors: SPFC_E_INVAL (null pointer, r_shift not finite, shifted r not positive),
 * SPFC_E_DEVICE. */
int spfc_batch_reset(spfc_batch* b, const double* const* phi_dev, const double* r_shift);
/* Every member's newest field into out_dev[member] (device, n_z x n_y x n_x, x fastest,
 * dtype SPFC_FP64 or SPFC_FP32): spfc_batch_get_phi for all members, with one launch
 * per transform pass for every 64 members of a grid size.  Queued on the batch's
 * stream, does not synchronize.  Errors: SPFC_E_INVAL (null pointer, dtype),
 * SPFC_E_DEVICE. */
int spfc_batch_get_phi_all(spfc_batch* b, void* const* out_dev, int dtype);
/* Energies of every member's current state (out: one entry per member) from one query
 * pass per class.  Returns SPFC_E_NONFINITE if any member's NONFINITE flag is set (the
 * entries are still filled).  Synchronizes. */
int spfc_batch_energies(spfc_batch* b, spfc_energy_t* out);
/* Free the host side of the batch.  Does not touch caller memory. */
int spfc_batch_destroy(spfc_batch* b);

/* ---------------------------------------------------------------- allocation-free run
 * For callers that cannot allocate device memory (code in tight serving loops, harnesses
 * that forbid hipMalloc): one whole run in a single call whose workspace is an array of
 * SPFC_NOALLOC_BYTES bytes that the library itself holds on each device it runs on
 * (allocated with the library's code object, kept until the process ends).  The call
 * does what spfc_init (on that array) + spfc_step(dt, n) + spfc_get_phi + spfc_energy +
 * spfc_destroy do, with the same kernels and launch plan, so its results equal theirs
 * bit for bit.  It calls no hipMalloc, hipFree or other allocating routine.
 * phi0_dev: N_total doubles (x fastest), read only.  phi_out_dev: N_total values of
 * dtype SPFC_FP64 or SPFC_FP32 (may equal phi0_dev), receives phi^n.  energy_out (host,
 * may be null) receives the energies of phi^n as spfc_energy gives them.  hip_stream as
 * for spfc_init.  Synchronizes the stream before returning.
 * Every call on one device uses that device's one array: calls that overlap on a device
 * (other host threads, other streams) race and must be serialized by the caller.  Each
 * call clears what must start at zero, so no state carries over from an earlier call.
 * Errors: SPFC_E_INVAL (as spfc_init / spfc_step, null output, bad dtype),
 * SPFC_E_NOMEM (spfc_workspace_bytes of the grid and parameters above
 * SPFC_NOALLOC_BYTES: with the default history of 4096 records that admits 2-D FP64
 * grids up to 2^19 points, FP32 up to 1024^2, 3-D FP32 up to 128 x 128 x 64),
 * SPFC_E_DEVICE, SPFC_E_NONFINITE (energies with the sticky NONFINITE flag set; phi_out
 * and energy_out are still written). */
#define SPFC_NOALLOC_BYTES ((size_t)64 << 20)
int spfc_run_noalloc(const spfc_grid* grid, const spfc_params* params, const double* phi0_dev, double dt,
                     int64_t n, void* phi_out_dev, int dtype, spfc_energy_t* energy_out, void* hip_stream);

/* Static description of a status code. */
const char* spfc_strerror(int status);

/* Free the host context.  Does not touch caller memory. */
int spfc_destroy(spfc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SPFC_H */
