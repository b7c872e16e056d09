/*
 * fno.h -- C interface of the Fourier-neural-operator surrogate in
 * libttsh.so: forward, hand-written backward and Adam on MI355X (gfx950), with
 * BF16 weights and activations and FP32 accumulation on the matrix cores.
 *
 * Architecture (Fourier neural operator, Li et al., ICLR 2021): per-point
 * lift cin -> C; `layers` Fourier layers h <- act(S(h) + h W + b), where S
 * multiplies the retained modes k_x = 0..m-1, k_y = -m..m-1 of rfft2(h) by a
 * complex C x C matrix per mode and transforms back (irfft2), act = exact
 * GELU except after the last layer; projection C -> hidden -> GELU -> cout.
 * The surrogate advances a coarse velocity field (input: v_x, v_y, K) by a
 * fixed number of solver steps; training pairs come from the solver.
 *
 * Layouts: fields are channels-last float32 [B][H][W][c] on the device.
 * Parameters are exchanged as one float32 vector in this order:
 *   P_w [cin][C], P_b [C],
 *   for each layer: R real part [2m][m][C][C], R imaginary part [2m][m][C][C]
 *     (row q of the 2m retained k_y rows is k_y = q for q < m, q - 2m else;
 *     R[q][k_x][i][o] maps input channel i to output channel o),
 *     W [C][C], b [C],
 *   Q1_w [C][hidden], Q1_b [hidden], Q2_w [hidden][cout], Q2_b [cout].
 * Transforms: rfft2 unnormalised, irfft2 with 1/(HW).
 * Loss: mean over samples of ||y - t||_2 / ||t||_2.
 *
 * Errors: 0 or a negative TTSH_* code (ttsh.h); message via ttsh_last_error().
 * The library owns its device buffers; caller buffers are never retained.
 */
#ifndef FNO_H
#define FNO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fno_ctx fno_ctx;

/* Create a network and its training state for batches of up to max_batch
 * samples of H x W (H, W multiples of 16, 2m <= H, m <= W/2).  Parameters are
 * drawn from a seeded generator (set them with fno_set_params to match an
 * outside model).  stream: hipStream_t (NULL = default stream).            */
int fno_create(fno_ctx** out, int width, int modes, int layers, int cin, int cout, int hidden,
               int H, int W, int max_batch, uint64_t seed, void* stream);
void fno_destroy(fno_ctx* ctx);

/* Implementation switches (value 1 = on, the default; 0 = off), for
 * comparing the kernel paths against each other.  Both leave the network's
 * function unchanged; results may differ by BF16 rounding.
 * FNO_OPT_STAGED_GEMM: GEMM operands staged through LDS where the layout allows.
 * FNO_OPT_SPECIALIZED: kernels written for width 32 and 16 modes: each
 *   Fourier layer's 1x1 convolution, inverse k_x transform, bias and GELU
 *   fused with the next layer's k_x transform (W = 128), and the k_y
 *   transform and synthesis as one kernel each (H = 128); other shapes take
 *   the general GEMMs.
 * Returns TTSH_EINVAL for an unknown option. */
#define FNO_OPT_STAGED_GEMM 1
#define FNO_OPT_SPECIALIZED 2
/* FNO_OPT_TAIL_PROJ: with the specialized kernels (and hidden 128, at most 16
 * outputs, at most 4 in a training forward), the last Fourier layer's tail
 * (1x1 convolution, inverse k_x transform, bias) fused with the projection,
 * so that h_layers is formed on chip and written to memory only for the
 * training backward or the stage capture.  On by default; the same bits as
 * the unfused pair. */
#define FNO_OPT_TAIL_PROJ 4
/* FNO_OPT_CAPTURE: keep each stage's BF16 intermediates per layer (for
 * stage-level tests; buffers of a few times the activations, allocated on
 * the first use), read with fno_capture.  Off by default. */
#define FNO_OPT_CAPTURE 3
int fno_set_option(fno_ctx* ctx, int option, int value);

/* Items of fno_capture, BF16 values read back as float32 (n elements from the
 * start; layouts for B samples, C channels, m modes, P = B H W points):
 *   FNO_CAP_XB   the input as BF16 [P][cin]                    (layer ignored)
 *   FNO_CAP_H    h_l, l = 0..layers [P][C] (l = layers: the projection input)
 *                (every h_l of the last forward run with capture on)
 *   FNO_CAP_Z    pre-activation z_l of a non-last layer [P][C] (training forward)
 *   FNO_CAP_T1   k_x transform of h_l: [B][2m][H][C], rows k_x (real) then m + k_x
 *                (imaginary), unnormalised, e^{-i k_x x}
 *   FNO_CAP_G    retained modes F_l: [m][4m][B][C] (k_x; rows q < 2m real parts of
 *                k_y = q or q - 2m, rows 2m + q imaginary parts)
 *   FNO_CAP_O    mixed modes R_l F_l: [m][2m][B][2C] (k_x; k_y rows; real C then
 *                imaginary C)
 *   FNO_CAP_T2   k_y synthesis of O: [B][H][2m][C] (k_x real, m + k_x imaginary)
 *   backward, per layer l, from the last fno_backward:
 *   FNO_CAP_DZ   dl/dz_l [P][C];  FNO_CAP_BT1 its k_x transform with the
 *                inverse weights (1 or 2)/(HW), as T1;  FNO_CAP_GG its retained
 *                modes, as G;  FNO_CAP_GF their adjoint mix R_l^H, as O;
 *                FNO_CAP_BT2 the k_y synthesis of GF, as T2;  FNO_CAP_DH the
 *                gradient the layer hands down: dl/dh_l (l = 0), or
 *                dl/dh_l times GELU'(z_{l-1}) (= dl/dz_{l-1}, l > 0)
 *   FNO_CAP_DHL  dl/dh_layers from the projection [P][C]
 *   FNO_CAP_DY   dl/dy as the backward pass takes it, BF16 [P][cout] (no capture
 *                needed; the last fno_loss)                                    */
enum {
  FNO_CAP_XB = 0, FNO_CAP_H = 1, FNO_CAP_Z = 2, FNO_CAP_T1 = 3, FNO_CAP_G = 4, FNO_CAP_O = 5, FNO_CAP_T2 = 6,
  FNO_CAP_DZ = 10, FNO_CAP_BT1 = 11, FNO_CAP_GG = 12, FNO_CAP_GF = 13, FNO_CAP_BT2 = 14, FNO_CAP_DH = 15,
  FNO_CAP_DHL = 16, FNO_CAP_DY = 17
};
int fno_capture(fno_ctx* ctx, int what, int layer, float* out, int64_t n);

/* Number of float32 parameters (the length of the vectors below). */
int64_t fno_num_params(fno_ctx* ctx);

/* Host float32 vectors in the order above.  set also resets nothing else. */
int fno_set_params(fno_ctx* ctx, const float* params);
int fno_get_params(fno_ctx* ctx, float* params);
int fno_get_grads(fno_ctx* ctx, float* grads);

/* y [B][H][W][cout] = network(x [B][H][W][cin]); device float32 buffers,
 * 1 <= batch <= max_batch.  With train != 0 the activations needed by
 * fno_backward are kept.  Asynchronous on the context's stream.            */
int fno_forward(fno_ctx* ctx, const float* x, float* y, int batch, int train);

/* Relative-L2 loss of the last training forward's output y against target t
 * (device float32, same shape); writes the loss (synchronous) and keeps
 * dl/dy for fno_backward.                                                  */
int fno_loss(fno_ctx* ctx, const float* y, const float* t, int batch, double* loss);

/* fno_loss with another normaliser: loss = mean over samples of
 * ||y - t|| / ||t - ref|| (the relative error of the change from ref when y
 * and t are fields one step apart and ref is the earlier field), ref holding
 * the cout channels of sample s, pixel p at ref[(s*H*W + p)*ref_stride + c]
 * (e.g. the network's input, ref_stride = cin).  ref = NULL is fno_loss.   */
int fno_loss_ex(fno_ctx* ctx, const float* y, const float* t, const float* ref, int64_t ref_stride, int batch,
                double* loss);

/* Gradients of the loss with respect to every parameter (overwritten). */
int fno_backward(fno_ctx* ctx, int batch);

/* One Adam step (Kingma & Ba) on the float32 master parameters. */
int fno_adam_step(fno_ctx* ctx, float lr, float beta1, float beta2, float eps);

/* fno_forward with two options.  Output element (p, o) (p = point index over
 * the batch, o < cout) is written to y[p * y_pix_stride + o]; with
 * residual != 0 it is x[p * cin + o] + network(x)[p][o] (requires
 * cout <= cin: the network predicts the change of the first cout input
 * channels).  y may alias x (e.g. the velocity channels of the next step's
 * input): x is converted before any output is written, and each output
 * element reads only its own residual input.  fno_loss and fno_backward
 * treat the residual as part of the output (it has no parameters).        */
int fno_forward_ex(fno_ctx* ctx, const float* x, float* y, int64_t y_pix_stride, int residual, int batch,
                   int train);

/* Gather training samples: for s < n, pixel p < npix, channel c < nch:
 * dst[(s*npix + p)*dst_ch + c] = src[(idx[s]*npix + p)*src_ch + c]
 * (device float32 buffers, idx host int64 indices, all within src's
 * extent, which the caller guarantees).  Asynchronous; n <= max_batch.    */
int fno_gather(fno_ctx* ctx, float* dst, int64_t dst_ch, const float* src, int64_t src_ch, int nch,
               int64_t npix, const int64_t* idx, int n);

/* fno_gather of square samples (n_side x n_side pixels, n_side even) with a
 * symmetry of the square per sample, for training-set augmentation (the
 * equation is isotropic and has no handedness, so a rotated or reflected
 * solution is a solution; a mask centred on the grid centre stays a valid
 * mask): sym[s] in 0..7 is the element g of the dihedral group D4, r = g & 3
 * quarter turns counterclockwise followed, if g & 4, by the reflection
 * y -> -y, about the node (n_side/2, n_side/2) of the periodic grid (rows y,
 * columns x).  Destination node x' takes source node M_g^-1 x'; channels 0
 * and 1 are a vector (v_x, v_y) and are multiplied by M_g; other channels are
 * copied.  idx and sym are host arrays.  Synchronous; n <= max_batch.
 * TTSH_EINVAL for odd n_side or sym outside 0..7.                          */
int fno_gather_d4(fno_ctx* ctx, float* dst, int64_t dst_ch, const float* src, int64_t src_ch, int nch,
                  int n_side, const int64_t* idx, const int* sym, int n);

/* Add uniform noise amp * U[-1, 1) to channels 0..nch-1 of npix pixels of
 * x (device float32, pixel stride pix_stride); the noise is a counter-based
 * SplitMix64 stream of (seed, element index), reproducible for any launch
 * shape.  For training-time input perturbation.  Asynchronous.            */
int fno_perturb(fno_ctx* ctx, float* x, int64_t pix_stride, int nch, int64_t npix, float amp, uint64_t seed);

/* Relative L2 error per sample between device float32 fields laid out with
 * pixel strides: sample s, pixel p, channel c at y[(s*npix + p)*ys + c] and
 * t[(s*npix + p)*ts + c], c < nch;  out[s] = ||y_s - t_s|| / ||t_s|| (host,
 * synchronous, FP64 sums).                                                 */
int fno_sample_errors(const float* y, int64_t ys, const float* t, int64_t ts, int nch, int64_t npix,
                      int batch, double* out);

/* Batched strided GEMM on the matrix cores, exposed for testing (it takes
 * the LDS-staged path whenever the strides allow, as the network does):
 * C[b][i][j] = alpha sum_k A[b][i][k] B[b][k][j] with A, B bfloat16 (raw
 * uint16 storage) and C float32, all device pointers; element (i, k) of
 * batch b of A sits at A + b*sA + i*rA + k*cA (likewise B, C).  Synchronous. */
int fno_gemm_bf16(int batch, int M, int N, int K, float alpha, const uint16_t* A, int64_t sA,
                  int64_t rA, int64_t cA, const uint16_t* B, int64_t sB, int64_t rB, int64_t cB,
                  float* C, int64_t sC, int64_t rC, int64_t cC);

#ifdef __cplusplus
}
#endif

#endif /* FNO_H */
