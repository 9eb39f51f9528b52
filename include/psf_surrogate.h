/*
 * psf_surrogate.h -- training and building-block entry points of the learned
 * PSF surrogate in libbpm.so (inference: psf_surrogate_infer in bpm.h).
 *
 * The surrogate maps a local refractive-index patch around a point source
 * (dn [64][32][32], z y x, dx = dz = 0.2 um) and the source depth (slice index)
 * to the source's refocused PSF stack [32][32][32] (planes, y, x), the object
 * that the paper assembles by the 10^5 - 10^6 from multiplexed BPM runs
 * (abstract; main-text paragraphs on multiplexing and image formation).  The
 * paper itself has no learned component; the network is this library's own:
 *
 *   input  5 channels: dn / 0.05, the mask [z >= depth], the lateral
 *          coordinates cy = (y - 15.5) / 16, cx = (x - 15.5) / 16 and
 *          cy^2 + cx^2 (the source sits at the patch centre)  (zero-padded to 8)
 *   c1     3x3x3 conv, 32 channels, stride (2,2,2), ReLU       -> [32][16][16]
 *   c2-c4  3x3x3 conv, 32 channels, stride (2,1,1), ReLU       -> [4][16][16]
 *   d1     4x3x3 conv over the remaining depth, 64 ch, ReLU    -> [16][16] (2-D)
 *   up     nearest x2                                           -> [32][32]
 *   d2     3x3 conv, 32 channels = PSF planes, softplus         -> [32][32][32]
 *   head   mean of d1 over (y, x) -> linear -> softplus = predicted relative
 *          L2 error of the PSF
 *
 * BF16 operands (weights and activations) on the matrix cores with FP32
 * accumulation; FP32 master weights, gradients and Adam moments.  Loss per
 * batch: mean_n |psf - t|^2 / |t|^2 + lambda mean_n (err_pred - err_true)^2,
 * err_true = |psf - t| / |t| (not differentiated).
 *
 * Conventions as in bpm.h: device pointers, caller-owned memory, asynchronous
 * on hip_stream, BPM_* return codes.
 */
#ifndef PSF_SURROGATE_H
#define PSF_SURROGATE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Number of fp32 master parameters.  Order: the six conv weights [Co][Kp]
 * (layers c1 c2 c3 c4 d1 d2, K ordered (tap, channel), zero padding K -> Kp),
 * then the six biases [Co], then the error head's weights [64] and bias [1]. */
size_t psf_surrogate_param_count(void);

/* Geometry of layer 0..5 for one sample, as the 15 integers of the building
 * blocks below (N = 1).  BPM_ERR_INVALID_ARG for another layer number. */
int psf_surrogate_layer_geometry(int layer, int* geom_out);

/* Bytes of the inference weight blob (bf16 weights, fp32 biases and head,
 * constant tap tables; validated by a header). */
size_t psf_surrogate_weights_bytes(void);

/* Bytes of the training state (master parameters, gradients, Adam moments,
 * bf16 and transposed bf16 weights, tap tables). */
size_t psf_surrogate_state_bytes(void);

/* Bytes of workspace for a training step (training = 1) or an inference call
 * (training = 0; inference runs in chunks of at most 1024 samples). */
size_t psf_surrogate_workspace_size(int batch, int training);

/* Fills the training state from fp32 initial parameters (device
 * [param_count]); Adam moments start at zero. */
int psf_surrogate_train_init(void* state, const float* init_params, void* hip_stream);

/* One training step on a batch: forward, loss, backward and, when lr > 0, an
 * Adam update (beta 0.9 / 0.999, eps 1e-8) at 1-based step `step`.
 *   dn [batch][64][32][32], depth [batch], target [batch][32][32][32] (fp32).
 *   loss_out  device float[2]: the PSF term and the error-head term.
 *   err_true  device float[batch] (or NULL): |psf - t| / |t| per sample. */
int psf_surrogate_train_step(void* state, const float* dn, const float* depth,
                             const float* target, int batch, float lr, float err_weight,
                             int step, float* loss_out, float* err_true, void* workspace,
                             size_t workspace_bytes, void* hip_stream);

/* The gradient vector of the last train step (device fp32 [param_count]). */
int psf_surrogate_gradients(const void* state, float* grads_out, void* hip_stream);

/* The current master parameters (device fp32 [param_count]). */
int psf_surrogate_params(const void* state, float* params_out, void* hip_stream);

/* Writes the inference blob (psf_surrogate_weights_bytes) from the state. */
int psf_surrogate_export(const void* state, void* weights_blob, void* hip_stream);

/* Cuts the surrogate's input patches out of a dn volume:
 *   patches[s][z][y][x] = dn[z0 + z][(sy - 16 + y) mod ny][(sx - 16 + x) mod nx]
 * for z < 64, y, x < 32, with (sy, sx) = sources[s] (device int32 [n][2]) --
 * the same window as a 32 x 32 PSF crop of bpm_psf_readout.  dn: device
 * float32 [nz][ny][nx] with ny, nx >= 32 and z0 + 64 <= nz; patches: device
 * float32 [n][64][32][32], 16-byte aligned. */
int psf_extract_patches(const float* dn, int nz, int ny, int nx, int z0, const int* sources,
                        int n, float* patches, void* hip_stream);

/* Building blocks, exposed for parity tests against the convolution oracle.
 * geom: host int[15] = {N, D, H, W, Ci, Co, kd, kh, kw, sd, sh, sw, pd, ph, pw};
 * Ci and Co multiples of 8 and of 32 respectively (Ci a multiple of 32 for the
 * data gradient).  x: bf16 [N][D][H][W][Ci]; w: fp32 [Co][Kp] with
 * K = kd kh kw Ci ordered (tap, channel) and zero padding to Kp = 16 ceil(K/16)
 * (rounded to bf16 inside); y / dy: bf16 [N][Do][Ho][Wo][Co].
 *   epilogue 0: y_bf16 = bf16(ReLU(conv + bias));
 *   epilogue 1: z = conv + bias, y_f32 = softplus(z), both [N][Co][Ho][Wo] with Do = 1.
 *   backward: dx (bf16 like x, masked by xmask > 0 when xmask is not NULL),
 *   dw fp32 [Co][Kp], db fp32 [Co]; any output may be NULL. */
size_t psf_conv_workspace_size(const int* geom);
int psf_conv_forward(const void* x, const float* w, const float* bias, const int* geom,
                     int epilogue, void* y_bf16, float* y_f32, float* z_f32, void* workspace,
                     size_t workspace_bytes, void* hip_stream);
int psf_conv_backward(const void* x, const float* w, const void* dy, const void* xmask,
                      const int* geom, void* dx, float* dw, float* db, void* workspace,
                      size_t workspace_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PSF_SURROGATE_H */
