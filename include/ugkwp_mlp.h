/*
 * Dense-layer kernels of the learned warm start (BF16 matrix-core operands,
 * FP32 accumulation; gfx950).
 *
 * The method of the paper (arXiv 2607.09552) starts every run from a given
 * initial field and fixes the local time steps from it (Sec. IV, Eq. (33));
 * it says nothing about where that field comes from.  This library predicts
 * it: a coarse wave-only solve is upsampled and corrected by a multilayer
 * perceptron with GELU activations, whose forward pass, backward pass and
 * Adam update run on these entry points.  They are an addition to the
 * paper's method, not part of it.
 *
 * Conventions for every entry point:
 *   - all pointers are device pointers, allocated and owned by the caller;
 *     no entry point allocates, frees or synchronizes;
 *   - matrices are row-major; BF16 values are raw uint16 bit patterns
 *     (upper half of the IEEE FP32 encoding; conversions round to nearest
 *     even);
 *   - work is enqueued on `stream` (a hipStream_t; NULL is the null stream);
 *   - return 0 on success, -1 for invalid arguments (nothing is enqueued),
 *     -3 if the launch failed.
 */
#ifndef UGKWP_MLP_H
#define UGKWP_MLP_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* One layer: Z = A B^T + bias, Y = GELU(Z) if act else Z, with
 * GELU(z) = z Phi(z) (Phi the standard normal distribution function).
 *   A  [M x K] BF16 (rows: samples), B [N x K] BF16 (rows: output units),
 *   bias [N] FP32 or NULL.
 * Outputs, each optional (NULL skips it): Z [M x N] FP32, Y32 [M x N] FP32,
 * Y16 [M x N] BF16, YT16 [N x M] BF16 (Y transposed).
 * Requires M % 32 == 0, N % 32 == 0, K % 16 == 0. */
int ugkwp_mlp_layer(const uint16_t *A, const uint16_t *B, const float *bias, int64_t M, int64_t N, int64_t K,
                    int32_t act, float *Z, float *Y32, uint16_t *Y16, uint16_t *YT16, void *stream);

/* G [M x N] FP32 += A [M x K] B [N x K]^T (BF16 operands), with K split into
 * chunks of k_chunk reduced by FP32 atomics: the weight gradient
 * dW = dZ^T X, called with A = dZ^T [N_out x batch] and B = X^T
 * [N_in x batch].  The caller clears G first.  Summation order across chunks
 * is not fixed.  Requires M % 32 == 0, N % 32 == 0, K % 16 == 0,
 * k_chunk % 16 == 0. */
int ugkwp_mlp_gemm_acc(const uint16_t *A, const uint16_t *B, int64_t M, int64_t N, int64_t K, int64_t k_chunk,
                       float *G, void *stream);

/* Backward of the activation and the bias:
 *   dZ = dY * GELU'(Z) if act else dY    (dY, Z [M x N] FP32; Z unused without act)
 * written as BF16 dZ16 [M x N] and dZT16 [N x M]; db [N] FP32 += column sums
 * of dZ (the caller clears db first; summation order not fixed). */
int ugkwp_mlp_act_backward(const float *dY, const float *Z, int64_t M, int64_t N, int32_t act, uint16_t *dZ16,
                           uint16_t *dZT16, float *db, void *stream);

/* Adam step t >= 1 (Kingma and Ba, 2015) on FP32 parameters w [n] with first
 * and second moments m, v [n] and gradient g [n]:
 *   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
 *   w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * Writes the BF16 copy w16 [n] (optional) and, viewing w as a [n / cols x cols]
 * matrix, its BF16 transpose wT16 (optional).  Requires n % cols == 0. */
int ugkwp_mlp_adam(float *w, float *m, float *v, const float *g, int64_t n, int64_t cols, float lr, float beta1,
                   float beta2, float eps, int64_t t, uint16_t *w16, uint16_t *wT16, void *stream);

/* Inference of the whole network in one kernel, the activations kept in
 * registers between layers (32 samples per wavefront, four wavefronts per
 * block; each layer's weights are staged once per block in LDS: 128 KiB).  Supported widths:
 * 32 -> 256 -> 256 -> 256 -> 32 (n_layers = 4), hidden layers with GELU,
 * the last linear; each activation is rounded to BF16 before the next layer,
 * as in ugkwp_mlp_layer.
 *   X [M x 32] BF16 inputs, M % 32 == 0;
 *   Wf[l]: layer l's weights packed by ugkwp_mlp_pack (permuted = 0 for
 *   l = 0, 1 for the others); bias[l] [widths[l+1]] FP32;
 *   Y [M x 32] FP32 outputs.
 * The pointer arrays Wf and bias are host arrays of device pointers. */
int ugkwp_mlp_forward(const uint16_t *X, int64_t M, int32_t n_layers, const int32_t *widths, const uint16_t *const *Wf,
                      const float *const *bias, float *Y, void *stream);

/* Weights W [out x in] FP32 (out % 32 == 0, in % 16 == 0) as BF16 in the
 * fragment order of ugkwp_mlp_forward:
 *   Wf[((t S + s) 64 + lane) 8 + e] = W[32 t + lane % 32][k],  S = in / 16,
 * with k = 16 s + 8 (lane / 32) + e (permuted = 0) or
 * k = 16 s + 8 (e / 4) + 4 (lane / 32) + e % 4 (permuted = 1: the order in
 * which a layer's outputs sit in the lanes). */
int ugkwp_mlp_pack(const float *W, int64_t out, int64_t in, int32_t permuted, uint16_t *Wf, void *stream);

/* BF16 copies of an FP32 matrix w [n / cols x cols]: w16 (same layout) and
 * wT16 (transposed), either optional but not both NULL. */
int ugkwp_mlp_to_bf16(const float *w, int64_t n, int64_t cols, uint16_t *w16, uint16_t *wT16, void *stream);

/* Loss gradient of the mean squared error
 *   L = sum_{r < M, c < n_out} (Y[r][c] - T[r][c])^2 / (M n_out)
 * for Y [M x N] FP32 (only the first n_out <= N columns are fitted) and
 * targets T [M x n_out] FP32: dY [M x N] = scale (Y - T) in the fitted
 * columns (scale = 2 / (M n_out) gives dL/dY), 0 elsewhere.  If loss is not
 * NULL, the sum of squares is added to it (the caller clears it). */
int ugkwp_mlp_mse_grad(const float *Y, const float *T, int64_t M, int64_t N, int64_t n_out, float scale, float *dY,
                       float *loss, void *stream);

/* One case of the warm start: the flow parameters the network is conditioned
 * on and the reference state the fields are normalized by. */
typedef struct {
  double Ma, Kn, Tw;            /* Mach and Knudsen numbers, wall temperature */
  double rho_inf, U_inf, T_inf; /* free stream */
  double R;                     /* gas constant */
  int32_t D;                    /* internal degrees of freedom */
} ugkwp_ws_case;

/* Feature rows of a fine O-grid of nft x nfr cells (cell (I, J), I the
 * angular index, at row J nft + I) from the converged fields of a coarse
 * wave-only solve of the same case on an nct x ncr O-grid whose nodes are
 * every (nft/nct)-th angular and (nfr/ncr)-th radial node of the fine one.
 *   Wc [ncr nct x 4] FP64 conservative coarse fields (device).
 * Row columns (BF16): 0-3 the coarse normalized primitives (ln rho/rho_inf,
 * u/U_inf, v/U_inf, ln T/T_inf) interpolated bilinearly in cell-index space
 * at x = (I + 1/2) nct/nft - 1/2 (periodic) and y = (J + 1/2) ncr/nfr - 1/2
 * (clamped to [0, ncr - 1]); 4-6 (Ma - 12.5)/7.5, (ln Kn - c)/h with
 * c = (ln 0.005 + ln 0.2)/2, h = ln(40)/2, and (T_w - 0.3)/0.2; 7-14
 * sin, cos(2 pi k s) for k = 1..4, s = (I + 1/2)/nft; 15 2 r - 1 and 16-21
 * sin, cos(pi k r) for k = 1..3, r = (J + 1/2)/nfr; 22-31 zero.  Rows from
 * nft nfr up to `rows` (a multiple of 32) are zero.
 * Outputs: X16 [rows x 32] BF16; XT16 [32 x rows] BF16 (optional); P32
 * [nft nfr x 4] FP32 the interpolated primitives (optional). */
int ugkwp_ws_features(const double *Wc, int32_t nct, int32_t ncr, int32_t nft, int32_t nfr,
                      const ugkwp_ws_case *c, int64_t rows, uint16_t *X16, uint16_t *XT16, float *P32, void *stream);

/* Initial field from the network output Y (rows of ldy >= 4 floats, columns
 * 0-3 the correction) and the interpolated primitives P32 [n x 4]:
 * p = P32 + Y[:, 0:4]; W [n x 4] FP64 = (rho, rho u, rho v, rho E) with
 * rho = rho_inf e^p0, u = U_inf p1, v = U_inf p2, T = T_inf e^p3 and
 * rho E = rho (u^2 + v^2)/2 + (3 + D) rho R T / 2. */
int ugkwp_ws_decode(const float *Y, int64_t ldy, const float *P32, int64_t n, const ugkwp_ws_case *c, double *W,
                    void *stream);

#ifdef __cplusplus
}
#endif
#endif
