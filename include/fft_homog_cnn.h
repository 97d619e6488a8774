/*
 * fft_homog_cnn.h -- C ABI of the voxel-CNN stiffness surrogate (MI355X, gfx950).
 *
 * A learned stand-in for the homogenized stiffness of section 3.3 of Pundir & Kammer
 * (arXiv:2408.03804): the solver of fft_homog.h produces the training data (the
 * 21 independent components of the 6x6 tangent of two-phase cells), this library
 * trains and evaluates the network, and the caller falls back to the solver for
 * samples that fft_homog_cnn_check() rejects.
 *
 * Network (channels-last activations, bf16 operands, fp32 accumulation on the matrix cores):
 *   a_0 = phase indicator (u8 0/1) of an n^3 cell
 *   a_l = gelu(conv_l(a_{l-1}) + b_l), l = 1..4;  conv_l: 3x3x3 taps, stride 2, periodic wrap:
 *         out[b, o, co] = sum_t sum_ci W_l[co][t][ci] a[b, (2 o + t - 1) mod m, ci]
 *         (t = (tz, ty, tx) in {0,1,2}^3, tz slowest)
 *   g   = voxel mean of a_4;  h = gelu([g, feat] W_5^T + b_5);  y = h W_6^T + b_6
 *   gelu(x) = x Phi(x) (erf form).  Loss: mean squared error over batch and outputs.
 * Parameters: one flat f32 vector in the order W_1, b_1, ..., W_4, b_4, W_5, b_5, W_6, b_6 with
 * W_l as [c_l][27][c_{l-1}], W_5 as [hidden][c_4 + n_feat], W_6 as [n_out][hidden].
 *
 * All buffers are device memory unless stated; every call is enqueued on the handle's stream
 * and returns after it has completed.  Status codes are those of fft_homog.h.
 */
#ifndef FFT_HOMOG_CNN_H
#define FFT_HOMOG_CNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fft_homog_cnn_desc {
  int n;            /* cell edge in voxels: a multiple of 16, 16..128 */
  int channels[5];  /* channels[0] = 1, then the widths of the four conv blocks (each 1..1024) */
  int hidden;       /* width of the hidden MLP layer (1..4096) */
  int n_feat;       /* scalar features per sample appended to the pooled features (0..32) */
  int n_out;        /* outputs per sample (1..4096) */
  int max_batch;    /* most samples per call (>= 1, max_batch (n/2)^3 < 2^31) */
} fft_homog_cnn_desc;

typedef struct fft_homog_cnn fft_homog_cnn_t;

/* Number of f32 parameters of the network.  Host only; EINVAL for an invalid descriptor. */
int fft_homog_cnn_param_count(const fft_homog_cnn_desc* d, size_t* count);

/* Device workspace bytes for a handle (parameters, Adam moments, gradients, activations of
 * max_batch samples).  Host only. */
int fft_homog_cnn_workspace_size(const fft_homog_cnn_desc* d, size_t* bytes);

/* Create a handle on a caller-owned, 256-byte aligned workspace of at least workspace_size
 * bytes (never freed by the library) and a hipStream_t (NULL: default stream). */
int fft_homog_cnn_create(const fft_homog_cnn_desc* d, void* dev_workspace, size_t bytes,
                         void* hip_stream, fft_homog_cnn_t** out);

/* Copy parameters in (device f32[param_count]); resets the Adam moments and step count. */
int fft_homog_cnn_set_params(fft_homog_cnn_t* h, const float* params);
/* Copy the current parameters out (device f32[param_count]). */
int fft_homog_cnn_get_params(fft_homog_cnn_t* h, float* params);

/* Forward pass of `batch` samples (1..max_batch).
 *   phase      u8[batch][n^3], layout [z][y][x], values 0 or 1 (others EINVAL, checked on device)
 *   feat       f32[batch][n_feat] (NULL allowed when n_feat == 0)
 *   out_scale  f32[batch] or NULL: out[b][:] is multiplied by out_scale[b]
 *   out_offset f32[batch][n_out] or NULL: then added, out = out_offset + out_scale * y
 *   out        f32[batch][n_out] */
int fft_homog_cnn_forward(fft_homog_cnn_t* h, const uint8_t* phase, const float* feat,
                          const float* out_scale, const float* out_offset, float* out, int batch);

/* Forward and backward pass: *loss (host) = mean over batch and outputs of (y - target)^2,
 * target f32[batch][n_out]; the gradient with respect to the flat parameters is kept in the
 * workspace for fft_homog_cnn_adam_step and, if grad is not NULL, copied to grad
 * (device f32[param_count]). */
int fft_homog_cnn_loss_grad(fft_homog_cnn_t* h, const uint8_t* phase, const float* feat,
                            const float* target, int batch, float* loss, float* grad);

/* One Adam step (Kingma & Ba, with bias correction) on the last gradient:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr mhat / (sqrt(vhat) + eps). */
int fft_homog_cnn_adam_step(fft_homog_cnn_t* h, float lr, float beta1, float beta2, float eps);

/* Error indicator of predicted stiffnesses, per sample (ok[b] = 1 passes, 0 fails):
 *   C (f32[batch][21], upper triangle row by row of the 6x6 Voigt tangent with engineering
 *   shear) must be positive definite and lie between the Reuss and Voigt bounds of its cell
 *   up to a slack s = tol |C_Voigt|_F (Frobenius norm): C_Voigt - C + s I and C - C_Reuss + s I
 *   positive definite, the bounds taken from
 *   the phase volume fractions of phase (u8[batch][n^3]) and the isotropic phase moduli
 *   lam_mu (f32[batch][2][2] = (lam, mu) of phase 0 and phase 1); and feat[b][0] must lie
 *   in [feat_lo, feat_hi] (the range seen in training).
 *   C2 (nullable, f32[batch][21]): the prediction of a second, independently trained network.
 *   C is then replaced in place by (C + C2) / 2, the tests above apply to that mean, and the
 *   spread |C - C2| / |(C + C2) / 2| (2-norms over the 21 components) must not exceed
 *   max_spread.
 *   spread_out (nullable, f32[batch]) receives that spread per sample (0 without C2), the
 *   statistic a caller calibrates max_spread on (held-out samples with known tangents). */
int fft_homog_cnn_check(fft_homog_cnn_t* h, const uint8_t* phase, const float* lam_mu,
                        const float* feat, float* C, const float* C2, int batch, float tol,
                        float feat_lo, float feat_hi, float max_spread, int* ok, float* spread_out);

/* Device time (ms, HIP events) of the last forward and of the last loss_grad call. */
int fft_homog_cnn_last_ms(const fft_homog_cnn_t* h, double* forward_ms, double* train_ms);

void fft_homog_cnn_destroy(fft_homog_cnn_t* h);

/* C[z][m][n] = sum over the z-th split of k of A(m, k) B(n, k) (bf16 operands, fp32 sums) on the
 * matrix cores; A(m, k) = A[m * sam + k * sak], B(n, k) = B[n * sbn + k * sbk] with sak == 1 or
 * sam == 1 (likewise for B); splits = 1..1024 equal ranges of k.  Test entry point of the GEMM
 * behind every layer. */
int fft_homog_cnn_debug_gemm(fft_homog_cnn_t* h, int M, int N, int K, const uint16_t* A, long long sam,
                             long long sak, const uint16_t* B, long long sbn, long long sbk, float* C,
                             int splits);

#ifdef __cplusplus
}
#endif

#endif /* FFT_HOMOG_CNN_H */
