/*
 * lbnn.h -- C ABI of the warm-start network for the axisymmetric lattice
 * Boltzmann solver (include/lbaxi.h): a 4-level convolutional U-Net that maps
 * per-node geometry / parameter features of a lattice to its steady macroscopic
 * fields (rho, u_z, u_r, u_theta, T), trained and run with hand-written gfx950
 * kernels (BF16 MFMA with FP32 accumulation).  Its prediction seeds the
 * populations at equilibrium (lbaxi_seed, which follows Eqs. 6 and 54 of
 * Li, He, Tang, Tao, arXiv:1003.0282); the lattice Boltzmann run to the
 * Eq. (57) residual stays the measure of its error.  The network itself is not
 * part of the paper.
 *
 * Network (tensors NHWC, H = nr rows along r, W = nz columns along z):
 *   encoder level l = 0..3, widths c_l:  sp(conv3x3) twice -> e_l,
 *                                         2x2 average pool between levels;
 *   decoder l = 2, 1, 0: concat(nearest 2x upsample of the level below, e_l)
 *                        -> sp(conv3x3) twice -> d_l;
 *   head: 1x1 convolution d_0 -> c_out channels; loss: mean squared error;
 *   sp(v) = log(1 + e^v) (softplus), whose derivative 1 - e^(-sp) the
 *   backward pass takes from the stored activation.
 * 3x3 convolutions use zero "same" padding and weights W[tap][c_in][c_out],
 * tap = (dy + 1) * 3 + (dx + 1): out[y][x] = sum in[y + dy][x + dx] W[tap].
 * Parameters are FP32 masters (flat, in the order e0a.W, e0a.b, e0b.W, e0b.b,
 * e1a ... e3b, d2a, d2b, d1a, d1b, d0a, d0b, head.W [c0][c_out], head.b);
 * the kernels read BF16 copies; activations and their gradients are BF16;
 * every contraction accumulates in FP32; Adam keeps FP32 moments.
 *
 * Ownership and errors follow include/lbaxi.h: the caller provides one
 * device workspace (>= lbnn_workspace_bytes, 256-byte aligned) and a HIP
 * stream; the library allocates no device memory; statuses are lbaxi_status.
 */
#ifndef LBNN_H
#define LBNN_H

#include <stddef.h>
#include <stdint.h>

#include "lbaxi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t H, W;         /* image size; both multiples of 8 */
  int32_t c_in;         /* input channels, <= 16 */
  int32_t c_out;        /* output channels, <= 8 */
  int32_t widths[4];    /* channel widths, multiples of 32 in 32..256 */
  int32_t max_batch;    /* largest batch passed to forward/backward;
                           max_batch * H * W < 2^22 */
} lbnn_desc;

typedef struct lbnn_s lbnn_t;

lbaxi_status lbnn_workspace_bytes(const lbnn_desc* d, size_t* bytes);
lbaxi_status lbnn_create(const lbnn_desc* d, void* d_workspace, size_t bytes, void* hip_stream,
                         lbnn_t** out);
void lbnn_destroy(lbnn_t* h);

/* Number of FP32 parameters (flat layout above). */
lbaxi_status lbnn_param_count(const lbnn_t* h, int64_t* n);
/* Copy FP32 parameters in / out (device pointers, flat layout). */
lbaxi_status lbnn_set_params(lbnn_t* h, const float* d_params);
lbaxi_status lbnn_get_params(lbnn_t* h, float* d_params);

/* Forward pass on a batch: d_x [batch][H][W][c_in] FP32 -> d_y
 * [batch][H][W][c_out] FP32 (either may be the caller's).  Keeps the
 * activations for a following lbnn_backward.  Asynchronous. */
lbaxi_status lbnn_forward(lbnn_t* h, const float* d_x, float* d_y, int32_t batch);

/* Backward pass of loss = mean((y - target)^2) for the batch of the last
 * forward: FP32 parameter gradients stay in the workspace (and are copied
 * to d_grads when non-NULL, flat layout); host_loss (may be NULL) receives
 * the loss and makes the call synchronous. */
lbaxi_status lbnn_backward(lbnn_t* h, const float* d_target, float* d_grads, double* host_loss);

/* Adam update (bias-corrected, step counter kept by the handle) with the
 * gradients of the last backward. */
lbaxi_status lbnn_adam(lbnn_t* h, float lr, float beta1, float beta2, float eps);

/* Forward + backward + Adam. */
lbaxi_status lbnn_train_step(lbnn_t* h, const float* d_x, const float* d_target, int32_t batch,
                             float lr, double* host_loss);

/* Network output -> solver fields: channel k of d_y [batch][H][W][c_out],
 * optionally low-passed, times host_scale[k] plus host_offset[k], is written
 * to d_fields[k] (a packed [batch][H][W] float field; NULL skips it), for k <
 * c_out.  smooth = 1 applies the separable (1, 2, 1)/4 filter along H and W
 * (edge values repeated), which removes the checkerboard (Nyquist) component
 * of a prediction; smooth = 0 copies.  host_scale, host_offset and d_fields
 * are host arrays of c_out entries. */
lbaxi_status lbnn_to_fields(lbnn_t* h, const float* d_y, int32_t batch, const float* host_scale,
                            const float* host_offset, int32_t smooth, float* const* d_fields);

/* Self-test of the BF16 MFMA accumulator layout the convolution kernels
 * rely on: multiplies known 32x16 by 16x32 matrices on the device and
 * compares every output; *host_mismatches receives the count (0 = pass).
 * d_counter is 4 bytes of caller-owned device memory.  Synchronises
 * hip_stream. */
lbaxi_status lbnn_mfma_selftest(int32_t* d_counter, void* hip_stream, int32_t* host_mismatches);

/* Text of the most recent lbnn error on the calling thread. */
const char* lbnn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBNN_H */
