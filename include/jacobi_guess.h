/*
 * jacobi_guess.h -- C-ABI of the learned initial guess for the Jacobi solver
 * of jacobi.h (libjacobi, gfx950).
 *
 * The Jacobi method (Sect. 1.1 of Wittmann et al. 2010) converges from any
 * starting field; this network maps the six boundary faces of an n^3 problem
 * to a starting interior field, trained on converged solutions produced by
 * the solver.  The network is a small 3D U-Net:
 *   - input: 16 channels per interior cell = the six face values at the
 *     cell's projections (faces i=0, i=n+1, j=0, j=n+1, k=0, k=n+1), the
 *     three centred coordinates x/(n+1) - 1/2, the face blend b, 6 zeros;
 *     b = sum_f g_f w_f / sum_f w_f with w_f = 1/(distance to face f);
 *   - `levels` resolutions n, n/2, ...; per encoder level two 3x3x3 conv +
 *     ReLU, then a stride-2 3x3x3 conv + ReLU down; per decoder level a
 *     nearest x2 upsampling added to the encoder output of that level, then
 *     two 3x3x3 conv + ReLU; a 1x1x1 head to one output channel, added to
 *     b (the network predicts a correction to the blend);
 *   - 16 channels everywhere, zero padding, BF16 weights and activations,
 *     FP32 accumulation (MFMA), FP32 master parameters and gradients.
 * Flat FP32 parameter vector, in this order: for every conv layer (enc0_a,
 * enc0_b, down0, enc1_a, ..., enc{L-1}_b, dec{L-2}_a, dec{L-2}_b, ...,
 * dec0_b) its weights [27][Cout][Cin] (tap t = (dz+1)*9 + (dy+1)*3 + (dx+1))
 * then its 16 biases; then the head's 16 weights and 1 bias.
 *
 * All device buffers are caller-owned.  Functions return 0 or a negative
 * jacobi_status (jacobi.h) and never abort; launches are asynchronous on the
 * stream given at creation.
 */
#ifndef JACOBI_GUESS_H
#define JACOBI_GUESS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jg_net_s jg_net;

/* Number of FP32 parameters of a `levels`-level network (levels 2..6). */
int jg_param_count(int32_t levels, int64_t *count);

/* Workspace bytes for edge n (n divisible by 2^(levels-1), n >= 2^(levels-1)). */
int jg_workspace_size(int64_t n, int32_t levels, size_t *bytes);

/* params, grads, adam_m, adam_v: device FP32 vectors of jg_param_count
 * entries (grads/m/v may be NULL for inference only).  workspace: 256-byte
 * aligned device memory of jg_workspace_size bytes. */
int jg_create(int64_t n, int32_t levels, float *params, float *grads,
              float *adam_m, float *adam_v, void *workspace,
              size_t workspace_bytes, void *stream, jg_net **out);

/* Forward pass on a dense (n+2)^3 FP64 box (only its faces are read).
 * `out` (n^3 FP32, may be NULL) receives the network output. */
int jg_forward(jg_net *h, const double *box, float *out);

/* After jg_forward: MSE loss against `target` (n^3 FP32) and backward pass;
 * parameter gradients are ADDED to `grads`.  If `loss` is non-NULL the
 * stream is synchronized and the loss written to it. */
int jg_backward(jg_net *h, const float *target, double *loss);

/* Weight W >= 0 of an extra loss term used by jg_backward from the next call
 * on: loss = mean((out-target)^2) + W * sum_m a_m^2, where a_m is the mean of
 * (out - target) * v_m over the interior and v_m(i,j,k) =
 * sin(pi p i/(n+1)) sin(pi q j/(n+1)) sin(pi r k/(n+1)) for p,q,r in {1,2}
 * (the eight discrete sine modes the Jacobi iteration of Sect. 1.1 damps
 * slowest; not a quantity of the paper).  0 (the default) is plain MSE.
 * JACOBI_EINVAL for a null handle or a weight outside [0, 1e12]. */
int jg_set_low_mode_weight(jg_net *h, double weight);

int jg_zero_grads(jg_net *h);

/* Adam step on params with grads (bias-corrected, step >= 1). */
int jg_adam(jg_net *h, float lr, float beta1, float beta2, float eps,
            int64_t step);

/* Writes the last forward output into the interior of a dense (n+2)^3 FP64
 * box (the solver's initial field); the boundary is left untouched. */
int jg_write_guess(jg_net *h, double *box);

/* The non-learned comparison guess: writes the face blend b (above) of the
 * box's own faces into the interior of the dense (n+2)^3 FP64 `box`. */
int jg_write_blend(jg_net *h, double *box);

int jg_destroy(jg_net *h);

/* ---- single convolution layers --------------------------------------------
 * The 3x3x3 convolutions of the network (16 -> 16 channels, zero padding 1,
 * stride 1 or 2), run by the same kernels as jg_forward / jg_backward on
 * caller-owned device buffers, so that their FP32 accumulators can be
 * checked on given BF16 operands.  x: [d][d][d][16] bfloat16 bit patterns
 * (channel last); w: [27][Cout][Cin] bfloat16, tap t = (dz+1)*9 + (dy+1)*3 +
 * (dx+1); d >= 1 and divisible by the stride; the output edge is d/stride.
 * Asynchronous on `stream`.  Errors: JACOBI_EINVAL (null pointer, d, stride),
 * JACOBI_EWORKSPACE, JACOBI_EHIP. */

/* Workspace bytes (256-byte aligned) the backward layer calls need. */
int jg_conv3_workspace_size(int64_t d, int32_t stride, size_t *bytes);

/* y[o][co] = bias[co] + sum_t sum_ci w[t][co][ci] x[stride*o + d_t][ci]:
 * [d/stride]^3 x 16 FP32, before ReLU and before BF16 rounding. */
int jg_conv3_forward(const uint16_t *x, int64_t d, const uint16_t *w,
                     const float *bias, int32_t stride, float *y, void *stream);

/* dx[v][ci] = sum over taps t and outputs o with stride*o + d_t = v of
 * sum_co w[t][co][ci] bf16(dy[o][co]): [d]^3 x 16 FP32, overwritten; dy is
 * [d/stride]^3 x 16 FP32 and enters the products rounded to BF16. */
int jg_conv3_backward_data(const float *dy, int64_t d, const uint16_t *w,
                           int32_t stride, float *dx, void *workspace,
                           size_t workspace_bytes, void *stream);

/* grad[t*256 + co*16 + ci] += sum_o bf16(dy[o][co]) x[stride*o + d_t][ci]
 * and grad[27*256 + co] += sum_o dy[o][co] (FP32; 27*256 + 16 entries). */
int jg_conv3_backward_weight(const uint16_t *x, int64_t d, const float *dy,
                             int32_t stride, float *grad, void *workspace,
                             size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* JACOBI_GUESS_H */
