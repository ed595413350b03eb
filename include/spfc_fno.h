/*
 * spfc_fno.h - C ABI of the Fourier-neural-operator (FNO) surrogate that jumps an
 * SPFC run from phi(t) to phi(t + 50 dt), trained on trajectories of the SAV-BDF2
 * solver (include/spfc.h), whose plain step is its fallback and judge.
 *
 * Network (per sample; epsilon is the sample's model parameter):
 *   lifting     v0[c] = Lw[c][0] phi + Lw[c][1] epsilon + Lb[c]                  c < 32
 *   layer l<4   u[o]  = synth(mix_l(anal(v_l)))[o] + sum_i Pw_l[o][i] v_l[i] + Pb_l[o]
 *               v_{l+1} = gelu(u) (l < 3),  v_4 = u (l = 3)
 *   projection  h[k] = gelu(sum_c Q1[k][c] v_4[c] + q1[k])  (k < 64),
 *               out = sum_k Q2[k] h[k] + q2
 *   filter      out_f = synth(anal(out))  (the increment restricted to the retained modes:
 *               the SPFC dynamics leaves nothing above them in 50 steps, and bf16 noise
 *               there would raise the energy the fallback judges by)
 *   output      phi_pred = phi + out_f - mean(out_f)  (keeps the mean of phi, as the SPFC
 *               dynamics does: Theorem 2.1 of the scheme)
 * on an N x N grid (x contiguous), N in {64, 128, 256}.  Truncated transforms with the
 * retained modes kx in [0,16), ky in [0,16) u [N-16, N) (512 modes, mode index
 * m = kx * 32 + j, ky = j for j < 16, N - 32 + j otherwise):
 *   anal(v)[m]    = (1/N^2) sum_{y,x} v[y][x] exp(-2 pi i (kx x + ky y) / N)
 *   synth(U)[y][x] = sum_m b_kx Re(U[m] exp(+2 pi i (kx x + ky y) / N)), b = 1 (kx = 0), 2
 *   mix_l(V)[o][m] = sum_i V[i][m] (Wr_l + i Wi_l)[m][i][o]
 * gelu(z) = z Phi(z) (Phi: standard normal distribution function).
 *
 * Precision: activations v_l and pre-activations are stored as bfloat16; the complex
 * mixing runs on BF16 matrix cores with FP32 accumulation (operands V and W rounded to
 * bfloat16); transforms, pointwise layers, projection, reductions and gradients are
 * FP32; master weights and Adam moments FP32.
 *
 * Parameters: one FP32 vector, in this order (row-major arrays):
 *   Lw[32][2], Lb[32],
 *   for l = 0..3: Wr_l[512][32][32], Wi_l[512][32][32], Pw_l[32][32], Pb_l[32],
 *   Q1[64][32], q1[64], Q2[64], q2[1].
 * Loss: mean over samples and points of (phi_pred - target)^2.
 *
 * Conventions as in spfc.h: int status returns (SPFC_OK = 0, SPFC_E_INVAL = 1,
 * SPFC_E_NOMEM = 2, SPFC_E_DEVICE = 3), *_dev pointers are device memory, the caller
 * owns the workspace and the stream, no device allocation inside the library, one host
 * thread per context.  All calls are asynchronous on the context stream unless noted.
 */
#ifndef SPFC_FNO_H
#define SPFC_FNO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spfc_fno spfc_fno;

/* n: grid points per axis (64, 128 or 256); max_batch: samples per call (1..128);
 * train: 1 to also hold gradients, Adam moments and the activations backward needs. */
typedef struct {
    int n;
    int max_batch;
    int train;
} spfc_fno_shape;

/* Number of FP32 parameters (4,200,801 for the layout above, at any n). */
int spfc_fno_param_count(int64_t* count);

/* Bytes of device workspace for the shape. */
int spfc_fno_workspace_bytes(const spfc_fno_shape* shape, size_t* bytes);

/* Create a context; params_dev (param_count floats) is copied into the workspace
 * (synchronizes).  Errors: SPFC_E_INVAL (bad shape, null pointer, misaligned
 * workspace: 256 bytes), SPFC_E_NOMEM, SPFC_E_DEVICE. */
int spfc_fno_init(const spfc_fno_shape* shape, const float* params_dev, void* workspace_dev,
                  size_t workspace_bytes, void* hip_stream, spfc_fno** out);

/* phi_pred for `batch` samples: phi_dev [batch][n][n], eps_dev [batch], out_dev
 * [batch][n][n] (FP32, x fastest; out_dev may equal phi_dev only if the caller no
 * longer needs phi). */
int spfc_fno_forward(spfc_fno* f, int batch, const float* phi_dev, const float* eps_dev, float* out_dev);

/* Per-kernel timing of one forward pass (same inputs and output as spfc_fno_forward;
 * out_dev must not alias phi_dev). Each launch of the pass is issued `reps` (1..1000)
 * times back to back between two HIP events on the network's stream; the average
 * duration of one launch is accumulated per kernel role. On return *count holds the
 * number of roles that ran, and the first min(count, cap) entries of names (static
 * strings owned by the library), avg_ms (mean duration of one launch of that role, over
 * its launches in the pass), bytes (algorithmic HBM bytes of one launch: reads plus
 * writes of activations, partial transforms and spectra) and launches (launches of the
 * role in one pass) are filled. The output holds the forward result. Synchronises the
 * stream. Returns SPFC_E_INVAL for bad arguments. */
int spfc_fno_time_forward(spfc_fno* f, int batch, const float* phi_dev, const float* eps_dev,
                          float* out_dev, int reps, int cap, const char** names, double* avg_ms,
                          double* bytes, int* launches, int* count);

/* Loss and gradient for `batch` samples with targets target_dev [batch][n][n]:
 * loss_dev (1 float) and grad_dev (param_count floats) receive the mean squared error
 * and its gradient with respect to the parameters (needs train = 1). */
int spfc_fno_grads(spfc_fno* f, int batch, const float* phi_dev, const float* eps_dev,
                   const float* target_dev, float* loss_dev, float* grad_dev);

/* One Adam step (beta1 0.9, beta2 0.999, epsilon 1e-8, bias-corrected, learning rate lr)
 * on the loss of the batch; loss_dev receives the loss before the step (needs train = 1). */
int spfc_fno_train_step(spfc_fno* f, int batch, const float* phi_dev, const float* eps_dev,
                        const float* target_dev, float lr, float* loss_dev);

/* Copy the current FP32 parameters to params_dev (param_count floats). */
int spfc_fno_get_params(spfc_fno* f, float* params_dev);

/* Free the host context.  Does not touch caller memory. */
int spfc_fno_destroy(spfc_fno* f);

#ifdef __cplusplus
}
#endif

#endif /* SPFC_FNO_H */
