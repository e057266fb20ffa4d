// Dense layers of the warm-start network on the matrix cores (gfx950):
// BF16 operands, FP32 accumulation with v_mfma_f32_32x32x16_bf16.
//
// One kernel computes C[M x N] = A[M x K] * B[N x K]^T for row-major A and B
// (both contiguous along K, so a lane's eight operand values are one 16-byte
// load), either into a plain output with the layer epilogue (bias, GELU,
// BF16 copies, optionally transposed) or, split along K, accumulated into an
// FP32 output with atomics (the weight gradient, whose K is the batch).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ugkwp_mlp.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// case values of the feature map, parameters already normalized
struct WsCase {
  double ma_n, kn_n, tw_n, rho_inf, U_inf, T_inf, R;
  int D;
};

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// BF16 bits of an FP32 value, rounded to nearest even (gfx950's
// v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }

// Standard normal distribution function Phi(z) = (1 + erf(z / sqrt 2)) / 2 with
// erf from Abramowitz and Stegun 7.1.26 (|error| <= 1.5e-7, below FP32
// arithmetic noise at BF16 outputs): for x >= 0,
// erf x = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) e^{-x^2}, t = 1 / (1 + p x);
// odd in x.  About a dozen instructions instead of the library's erff.
__device__ __forceinline__ float phi_cdf(float z) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));  // v_rcp_f32, ~1 ulp
  float poly = fmaf(1.061405429f, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  const float e = 1.0f - poly * t * __expf(-x * x);  // erf(|z| / sqrt 2)
  return 0.5f + 0.5f * copysignf(e, z);
}

__device__ __forceinline__ float gelu(float z) { return z * phi_cdf(z); }

// d/dz z Phi(z) = Phi(z) + z phi(z), phi the standard normal density
__device__ __forceinline__ float gelu_grad(float z) {
  return phi_cdf(z) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

// Each wavefront computes one 32 x 32 tile of C over the K range
// [k_begin, k_end) (a multiple of 16).  Lane l holds A[row0 + l % 32][k + 8 (l / 32) .. + 7]
// and B[col0 + l % 32][same k]; the accumulator's element i of lane l is
// C[row0 + 8 (i / 4) + 4 (l / 32) + i % 4][col0 + l % 32].
__device__ __forceinline__ f32x16 tile_mma(const uint16_t *__restrict__ A, int64_t lda, const uint16_t *__restrict__ B,
                                           int64_t ldb, int64_t row0, int64_t col0, int64_t k_begin, int64_t k_end) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;
  const uint16_t *pa = A + (row0 + r) * lda + 8 * h;
  const uint16_t *pb = B + (col0 + r) * ldb + 8 * h;
  f32x16 acc = {};
  for (int64_t k = k_begin; k < k_end; k += 16) {
    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(pa + k);
    const bf16x8 b = *reinterpret_cast<const bf16x8 *>(pb + k);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// NB adjacent 32 x 32 tiles of C in one row band: one A fragment per k step
// serves NB matrix-core operations (register blocking); the k loop is
// unrolled so that later steps' loads are in flight during the current
// step's operations.  Each tile's operations run in the same k order as in
// tile_mma, so the results are the same bit for bit.
template <int NB, int KC>
__device__ __forceinline__ void tile_mma_nb(const uint16_t *__restrict__ A, int64_t lda,
                                            const uint16_t *__restrict__ B, int64_t ldb, int64_t row0, int64_t col0,
                                            int64_t Kr, f32x16 (&acc)[NB]) {
  // KC > 0: K known at compile time, the loop unrolled completely (all
  // operand loads can be issued ahead of the matrix-core operations)
  const int lane = threadIdx.x & 63;
  const int r = lane & 31, h = lane >> 5;
  const uint16_t *pa = A + (row0 + r) * lda + 8 * h;
  const uint16_t *pb = B + (col0 + r) * ldb + 8 * h;
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = f32x16{};
  auto step = [&](int64_t k) {
    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(pa + k);
    bf16x8 b[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(pb + 32 * j * ldb + k);
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b[j], acc[j], 0, 0, 0);
  };
  if constexpr (KC > 0) {
    // every operand fragment first, then the operations
    bf16x8 a[KC / 16], b[KC / 16][NB];
#pragma unroll
    for (int q = 0; q < KC / 16; ++q) {
      a[q] = *reinterpret_cast<const bf16x8 *>(pa + 16 * q);
#pragma unroll
      for (int j = 0; j < NB; ++j) b[q][j] = *reinterpret_cast<const bf16x8 *>(pb + 32 * j * ldb + 16 * q);
    }
    // keep the scheduler from sinking the loads back between the operations
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < KC / 16; ++q) {
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[q], b[q][j], acc[j], 0, 0, 0);
    }
  } else {
#pragma unroll 4
    for (int64_t k = 0; k < Kr; k += 16) step(k);
  }
}

// Layer: Z = A B^T + bias; with act, Y = GELU(Z) else Y = Z.  Writes Z (FP32,
// optional), Y as FP32 (optional), as BF16 (optional) and as transposed BF16
// [N x M] (optional).  Grid: (M / 32) x (N / (32 NB)) wavefronts, 4 per
// block; a wavefront takes NB adjacent column tiles.
template <int NB, int KC>
__global__ void __launch_bounds__(256, 2) k_layer(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B,
                                               const float *__restrict__ bias, int64_t M, int64_t N, int64_t K,
                                               int act, float *__restrict__ Z, float *__restrict__ Y32,
                                               uint16_t *__restrict__ Y16, uint16_t *__restrict__ YT16) {
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 6;
  const int64_t tiles_n = N / (32 * NB);
  if (wave >= (M / 32) * tiles_n) return;
  const int64_t row0 = (wave / tiles_n) * 32, col00 = (wave % tiles_n) * 32 * NB;
  f32x16 acc[NB];
  tile_mma_nb<NB, KC>(A, K, B, K, row0, col00, K, acc);
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int64_t col = col00 + 32 * j + (lane & 31);
    const float bc = bias ? bias[col] : 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int64_t row = row0 + 8 * (i / 4) + 4 * (lane >> 5) + (i % 4);
      const float z = acc[j][i] + bc;
      const float y = act ? gelu(z) : z;
      if (Z) Z[row * N + col] = z;
      if (Y32) Y32[row * N + col] = y;
      const uint16_t yb = f2bf(y);
      if (Y16) Y16[row * N + col] = yb;
      if (YT16) YT16[col * M + row] = yb;
    }
  }
}

// Weight gradient: G[M x N] += A B^T over K split into chunks of kc; one
// wavefront per (tile, chunk), FP32 atomics into G (cleared by the caller).
__global__ void __launch_bounds__(256) k_gemm_splitk(const uint16_t *__restrict__ A, const uint16_t *__restrict__ B,
                                                     int64_t M, int64_t N, int64_t K, int64_t kc,
                                                     float *__restrict__ G) {
  const int64_t wave = (blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x) >> 6;
  const int64_t tiles = (M / 32) * (N / 32);
  const int64_t chunks = (K + kc - 1) / kc;
  if (wave >= tiles * chunks) return;
  const int64_t t = wave % tiles, ch = wave / tiles;
  const int64_t tiles_n = N / 32;
  const int64_t row0 = (t / tiles_n) * 32, col0 = (t % tiles_n) * 32;
  const int64_t k0 = ch * kc, k1 = k0 + kc < K ? k0 + kc : K;
  const f32x16 acc = tile_mma(A, K, B, K, row0, col0, k0, k1);
  const int lane = threadIdx.x & 63;
  const int64_t col = col0 + (lane & 31);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int64_t row = row0 + 8 * (i / 4) + 4 * (lane >> 5) + (i % 4);
    atomicAdd(&G[row * N + col], acc[i]);
  }
}

// dZ = dY * GELU'(Z) (or dY without activation); writes dZ as BF16 [M x N]
// and transposed [N x M], and adds the column sums to db (cleared by the
// caller).  A block takes a tile of 64 rows x 32 columns: reads and the
// row-major write go along rows (32 consecutive columns), the transposed
// write goes through a padded LDS tile so that it runs along the 64 rows,
// and the column sums are reduced in LDS: one atomic per column per tile.
__global__ void __launch_bounds__(256) k_act_backward(const float *__restrict__ dY, const float *__restrict__ Z,
                                                      int64_t M, int64_t N, int act, uint16_t *__restrict__ dZ16,
                                                      uint16_t *__restrict__ dZT16, float *__restrict__ db) {
  __shared__ uint16_t tile[64][33];
  __shared__ float part[8][32];
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * 64, col0 = static_cast<int64_t>(blockIdx.y) * 32;
  const int c = threadIdx.x & 31, g = threadIdx.x >> 5;  // column, row group (8 rows apart)
  const int64_t col = col0 + c;
  float sum = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int r = g + 8 * k;
    const int64_t row = row0 + r;
    uint16_t b = 0;
    if (row < M && col < N) {
      const float gy = dY[row * N + col];
      const float v = act ? gy * gelu_grad(Z[row * N + col]) : gy;
      b = f2bf(v);
      dZ16[row * N + col] = b;
      sum += v;
    }
    tile[r][c] = b;
  }
  part[g][c] = sum;
  __syncthreads();
  if (threadIdx.x < 32 && col < N) {
    float s8 = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q) s8 += part[q][threadIdx.x];
    atomicAdd(&db[col], s8);
  }
  const int r = threadIdx.x & 63, q4 = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int cc = q4 + 4 * k;
    const int64_t row = row0 + r, cg = col0 + cc;
    if (row < M && cg < N) dZT16[cg * M + row] = tile[r][cc];
  }
}

// Adam (Kingma and Ba) on FP32 master weights w, moments m, v; step t >= 1;
// writes the BF16 copy and, for a matrix [R x C] (C > 1), its transpose.
__global__ void __launch_bounds__(256) k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                              const float *__restrict__ g, int64_t n, int64_t cols, float lr,
                                              float b1, float b2, float eps, float c1, float c2,
                                              uint16_t *__restrict__ w16, uint16_t *__restrict__ wT16) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  const uint16_t b = f2bf(wi);
  if (w16) w16[i] = b;
  if (wT16) {
    const int64_t rows = n / cols, r = i / cols, c = i % cols;
    wT16[c * rows + r] = b;
  }
}

// Loss gradient of the mean squared error over the first n_out of N output
// columns: dY = scale (Y - T) there, 0 in the padding; loss += sum (Y - T)^2
// (one atomic per wavefront).
__global__ void __launch_bounds__(256) k_mse_grad(const float *__restrict__ Y, const float *__restrict__ T,
                                                  int64_t M, int64_t N, int64_t n_out, float scale,
                                                  float *__restrict__ dY, float *__restrict__ loss) {
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  float sq = 0.0f;
  if (e < M * N) {
    const int64_t r = e / N, c = e % N;
    float g = 0.0f;
    if (c < n_out) {
      const float d = Y[e] - T[r * n_out + c];
      g = scale * d;
      sq = d * d;
    }
    dY[e] = g;
  }
  if (loss) {
    // one atomic per block: wavefront butterflies, then the four partials
    __shared__ float wsum[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]));
  }
}

// Normalized primitives (ln rho/rho_inf, u/U_inf, v/U_inf, ln T/T_inf) of a
// conservative 2D state with rho E = rho |U|^2 / 2 + (3 + D) rho R T / 2.
__device__ __forceinline__ void norm_prim(const double *w, const WsCase &c, double p[4]) {
  const double rho = w[0], u = w[1] / rho, v = w[2] / rho;
  const double T = (w[3] / rho - 0.5 * (u * u + v * v)) / (0.5 * (3 + c.D) * c.R);
  p[0] = log(rho / c.rho_inf);
  p[1] = u / c.U_inf;
  p[2] = v / c.U_inf;
  p[3] = log(T / c.T_inf);
}

// Feature rows of the fine O-grid (cell (I, J) at row J nft + I): columns 0-3
// the coarse normalized primitives interpolated bilinearly in cell-index
// space (periodic in the angular index, clamped in the radial one), 4-6 the
// normalized case parameters, 7-14 sin/cos(2 pi k s) (k = 1..4,
// s = (I + 1/2)/nft), 15 2 r - 1 and 16-21 sin/cos(pi k r) (k = 1..3,
// r = (J + 1/2)/nfr), 22-31 zero; rows from nft nfr to `rows` are zero.
__global__ void __launch_bounds__(256) k_ws_features(const double *__restrict__ Wc, int nct, int ncr, int nft,
                                                     int nfr, WsCase c, int64_t rows, uint16_t *__restrict__ X16,
                                                     uint16_t *__restrict__ XT16, float *__restrict__ P32) {
  const int64_t row = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (row >= rows) return;
  float f[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) f[k] = 0.0f;
  const int64_t nf = static_cast<int64_t>(nft) * nfr;
  if (row < nf) {
    const int I = static_cast<int>(row % nft), J = static_cast<int>(row / nft);
    double y = (J + 0.5) * ncr / nfr - 0.5;
    y = y < 0.0 ? 0.0 : (y > ncr - 1.0 ? ncr - 1.0 : y);
    int j0 = static_cast<int>(floor(y));
    if (j0 > ncr - 2) j0 = ncr - 2;
    const double b = y - j0;
    const double x = (I + 0.5) * nct / nft - 0.5;
    const int i0 = static_cast<int>(floor(x));
    const double a = x - i0;
    const int i0m = ((i0 % nct) + nct) % nct, i1m = (i0m + 1) % nct;
    double p00[4], p01[4], p10[4], p11[4];
    norm_prim(Wc + 4 * (static_cast<int64_t>(j0) * nct + i0m), c, p00);
    norm_prim(Wc + 4 * (static_cast<int64_t>(j0) * nct + i1m), c, p01);
    norm_prim(Wc + 4 * (static_cast<int64_t>(j0 + 1) * nct + i0m), c, p10);
    norm_prim(Wc + 4 * (static_cast<int64_t>(j0 + 1) * nct + i1m), c, p11);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double v = (1 - a) * (1 - b) * p00[k] + a * (1 - b) * p01[k] + (1 - a) * b * p10[k] + a * b * p11[k];
      f[k] = static_cast<float>(v);
      if (P32) P32[row * 4 + k] = static_cast<float>(v);
    }
    f[4] = static_cast<float>(c.ma_n);
    f[5] = static_cast<float>(c.kn_n);
    f[6] = static_cast<float>(c.tw_n);
    const double s = (I + 0.5) / nft, r = (J + 0.5) / nfr;
    constexpr double kPi = 3.141592653589793238;
#pragma unroll
    for (int k = 1; k <= 4; ++k) {
      f[5 + 2 * k] = static_cast<float>(sin(2.0 * kPi * k * s));
      f[6 + 2 * k] = static_cast<float>(cos(2.0 * kPi * k * s));
    }
    f[15] = static_cast<float>(2.0 * r - 1.0);
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
      f[14 + 2 * k] = static_cast<float>(sin(kPi * k * r));
      f[15 + 2 * k] = static_cast<float>(cos(kPi * k * r));
    }
  }
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const uint16_t b = f2bf(f[k]);
    X16[row * 32 + k] = b;
    if (XT16) XT16[k * rows + row] = b;
  }
}

// Initial field from the network output: p = P + Y[:, 0:4] (Y rows of ldy
// floats), rho = rho_inf e^p0, u = U_inf p1, v = U_inf p2, T = T_inf e^p3,
// written as conservative FP64 (rho, rho u, rho v, rho E).
__global__ void __launch_bounds__(256) k_ws_decode(const float *__restrict__ Y, int64_t ldy,
                                                   const float *__restrict__ P, int64_t n, WsCase c,
                                                   double *__restrict__ W) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  double p[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) p[k] = static_cast<double>(P[i * 4 + k]) + static_cast<double>(Y[i * ldy + k]);
  const double rho = c.rho_inf * exp(p[0]), u = c.U_inf * p[1], v = c.U_inf * p[2], T = c.T_inf * exp(p[3]);
  W[4 * i + 0] = rho;
  W[4 * i + 1] = rho * u;
  W[4 * i + 2] = rho * v;
  W[4 * i + 3] = 0.5 * rho * (u * u + v * v) + 0.5 * (3 + c.D) * rho * c.R * T;
}

// ---- whole-network forward with the activations in registers ----------
//
// Each wavefront pushes 32 samples through every layer.  A layer is computed
// transposed, D = W X^T (the MFMA's A operand a weight tile, its B operand the
// activations), so that lane l of the result holds sample l % 32 and outputs
// out0 + 8 (r / 4) + 4 (l / 32) + r % 4 of its tile (r = 0..15).  Those are
// exactly the eight values per lane of the next layer's B operand for two
// k-steps if the next layer's input features are taken in the matching order:
// k-step s, lane half h, slot e <-> feature 16 s + 8 (e / 4) + 4 h + e % 4.
// The weights are packed once (k_pack_frag) in that order and in fragment
// order, so a layer's weights are one contiguous array that a block copies
// to LDS with 16-byte loads, and a lane's A operand is one 16-byte LDS read.
// The first layer reads its inputs from memory in natural order.

// feature index of slot e of lane half h in k-step s
__host__ __device__ __forceinline__ int64_t frag_feature(int64_t s, int h, int e, int permuted) {
  return permuted ? 16 * s + 8 * (e / 4) + 4 * h + (e % 4) : 16 * s + 8 * h + e;
}

// Wf[((t * S + s) * 64 + lane) * 8 + e] = bf16(W[32 t + lane % 32][frag_feature(s, lane / 32, e)])
// for W [out x in] FP32, S = in / 16, t < out / 32.
__global__ void __launch_bounds__(256) k_pack_frag(const float *__restrict__ W, int64_t out, int64_t in,
                                                   int permuted, uint16_t *__restrict__ Wf) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= out * in) return;
  const int e = static_cast<int>(i % 8), lane = static_cast<int>((i / 8) % 64);
  const int64_t ts = i / 512, S = in / 16;
  const int64_t t = ts / S, s = ts % S;
  Wf[i] = f2bf(W[(32 * t + lane % 32) * in + frag_feature(s, lane / 32, e, permuted)]);
}

struct FusedNet {
  const uint16_t *W[4];  // packed fragments: layer 0 natural order, later layers permuted
  const float *b[4];
};

union Frag {
  bf16x8 v;
  uint16_t h[8];
};

// One layer on register activations: in [KS] k-steps -> acc [T] tiles,
// the accumulators starting from the bias (a lane's 16 outputs of a tile are
// four runs of four consecutive features: four 16-byte loads), the weight
// fragments read from the layer's copy in LDS (lane l's 16 bytes of a
// fragment are consecutive: conflict-free ds_read_b128).
template <int KS, int T>
__device__ __forceinline__ void layer_lds(const bf16x8 *__restrict__ lds, const float *__restrict__ bias,
                                          const Frag (&act)[KS], f32x16 (&acc)[T], int lane) {
  const int h = lane >> 5;
#pragma unroll
  for (int t = 0; t < T; ++t) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float4 b = *reinterpret_cast<const float4 *>(bias + 32 * t + 8 * g + 4 * h);
      acc[t][4 * g + 0] = b.x;
      acc[t][4 * g + 1] = b.y;
      acc[t][4 * g + 2] = b.z;
      acc[t][4 * g + 3] = b.w;
    }
  }
  const bf16x8 *w = lds + lane;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
#pragma unroll
    for (int t = 0; t < T; ++t)
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w[(t * KS + s) * 64], act[s].v, acc[t], 0, 0, 0);
  }
}

// The block's copy of one layer's packed fragments (n chunks of 16 bytes, a
// multiple of 64): each wavefront copies whole kilobytes with direct
// global-to-LDS loads (global_load_lds_dwordx4: lane l's 16 bytes land at
// the chunk's base + 16 l), all in flight at once and through no registers.
// The first barrier lets the previous layer's reads finish; the wait and the
// second barrier publish the copy.
__device__ __forceinline__ void stage_layer(const uint16_t *__restrict__ Wf, int n, bf16x8 *lds) {
  const bf16x8 *src = reinterpret_cast<const bf16x8 *>(Wf);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  for (int c = wv; c < n / 64; c += nw) __builtin_amdgcn_global_load_lds(src + c * 64 + lane, &lds[c * 64], 16, 0, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// GELU and BF16: the accumulators of T tiles become 2T k-steps of the next
// layer's operand
template <int T>
__device__ __forceinline__ void to_next(const f32x16 (&acc)[T], Frag (&act)[2 * T]) {
#pragma unroll
  for (int t = 0; t < T; ++t) {
#pragma unroll
    for (int r = 0; r < 16; ++r) act[2 * t + r / 8].h[r % 8] = f2bf(gelu(acc[t][r]));
  }
}

// widths K0 -> H -> H (NH - 1 times) -> NO.  A block of four wavefronts
// (128 rows) stages each layer's weights in LDS once (the H x H layer: 128 KiB
// of gfx950's 160 KiB), so the weights cross L2 once per block instead of once
// per wavefront, and the matrix cores wait on LDS instead of L2.
template <int K0, int H, int NH, int NO>
__global__ void __launch_bounds__(256) k_mlp_fused(const uint16_t *__restrict__ X, int64_t M, FusedNet net,
                                                  float *__restrict__ Y) {
  __shared__ bf16x8 lds[(H / 32) * (H / 16) * 64];
  const int lane = threadIdx.x & 63, sl = lane & 31, h = lane >> 5;
  const int64_t row0 = (static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6)) * 32;
  const bool active = row0 < M;  // M % 32 == 0: a wavefront's rows are all in or all out
  Frag xin[K0 / 16];
  Frag act[H / 16];
  if (active) {
#pragma unroll
    for (int s = 0; s < K0 / 16; ++s)
      xin[s].v = *reinterpret_cast<const bf16x8 *>(X + (row0 + sl) * K0 + 16 * s + 8 * h);
  }
  stage_layer(net.W[0], (H / 32) * (K0 / 16) * 64, lds);
  if (active) {
    f32x16 acc[H / 32];
    layer_lds<K0 / 16, H / 32>(lds, net.b[0], xin, acc, lane);
    to_next<H / 32>(acc, act);
  }
#pragma unroll
  for (int l = 1; l < NH; ++l) {
    stage_layer(net.W[l], (H / 32) * (H / 16) * 64, lds);
    if (active) {
      f32x16 acc[H / 32];
      layer_lds<H / 16, H / 32>(lds, net.b[l], act, acc, lane);
      to_next<H / 32>(acc, act);
    }
  }
  stage_layer(net.W[NH], (NO / 32) * (H / 16) * 64, lds);
  if (!active) return;
  f32x16 out[NO / 32];
  layer_lds<H / 16, NO / 32>(lds, net.b[NH], act, out, lane);
#pragma unroll
  for (int t = 0; t < NO / 32; ++t) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int o = 32 * t + 8 * g + 4 * h;
      float4 v;
      v.x = out[t][4 * g + 0];
      v.y = out[t][4 * g + 1];
      v.z = out[t][4 * g + 2];
      v.w = out[t][4 * g + 3];
      *reinterpret_cast<float4 *>(Y + (row0 + sl) * NO + o) = v;
    }
  }
}

// BF16 copies of an FP32 [rows x cols] matrix: w16 same layout, wT16 transposed.
__global__ void __launch_bounds__(256) k_to_bf16(const float *__restrict__ w, int64_t n, int64_t cols,
                                                 uint16_t *__restrict__ w16, uint16_t *__restrict__ wT16) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const uint16_t b = f2bf(w[i]);
  if (w16) w16[i] = b;
  if (wT16) wT16[(i % cols) * (n / cols) + i / cols] = b;
}

int64_t blocks_for_waves(int64_t waves) { return (waves + 3) / 4; }

bool case_ok(const ugkwp_ws_case *c) {
  return c && c->rho_inf > 0.0 && c->U_inf > 0.0 && c->T_inf > 0.0 && c->R > 0.0 && c->D >= 0 && c->Kn > 0.0;
}

WsCase make_case(const ugkwp_ws_case *c) {
  WsCase w;
  w.ma_n = (c->Ma - 12.5) / 7.5;
  const double lc = 0.5 * (log(0.005) + log(0.2)), lh = 0.5 * log(40.0);
  w.kn_n = (log(c->Kn) - lc) / lh;
  w.tw_n = (c->Tw - 0.3) / 0.2;
  w.rho_inf = c->rho_inf;
  w.U_inf = c->U_inf;
  w.T_inf = c->T_inf;
  w.R = c->R;
  w.D = c->D;
  return w;
}

}  // namespace

extern "C" {

int ugkwp_mlp_layer(const uint16_t *A, const uint16_t *B, const float *bias, int64_t M, int64_t N, int64_t K,
                    int32_t act, float *Z, float *Y32, uint16_t *Y16, uint16_t *YT16, void *stream) {
  if (!A || !B || M <= 0 || N <= 0 || K <= 0 || M % 32 || N % 32 || K % 16) return -1;
  // two column tiles per wavefront where N allows it; the network's inner
  // sizes (K = 32, 256) with the k loop unrolled completely
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = N % 64 == 0 ? 2 : 1;
  const unsigned blocks = static_cast<unsigned>(blocks_for_waves((M / 32) * (N / (32 * nb))));
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, s, A, B, bias, M, N, K, act, Z, Y32, Y16, YT16);
  };
  if (nb == 2) {
    if (K == 256) go(k_layer<2, 256>);
    else if (K == 32) go(k_layer<2, 32>);
    else go(k_layer<2, 0>);
  } else {
    if (K == 256) go(k_layer<1, 256>);
    else if (K == 32) go(k_layer<1, 32>);
    else go(k_layer<1, 0>);
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ugkwp_mlp_gemm_acc(const uint16_t *A, const uint16_t *B, int64_t M, int64_t N, int64_t K, int64_t k_chunk,
                       float *G, void *stream) {
  if (!A || !B || !G || M <= 0 || N <= 0 || K <= 0 || M % 32 || N % 32 || K % 16 || k_chunk <= 0 ||
      k_chunk % 16)
    return -1;
  const int64_t waves = (M / 32) * (N / 32) * ((K + k_chunk - 1) / k_chunk);
  hipLaunchKernelGGL(k_gemm_splitk, dim3(static_cast<unsigned>(blocks_for_waves(waves))), dim3(256), 0,
                     static_cast<hipStream_t>(stream), A, B, M, N, K, k_chunk, G);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ugkwp_mlp_act_backward(const float *dY, const float *Z, int64_t M, int64_t N, int32_t act, uint16_t *dZ16,
                           uint16_t *dZT16, float *db, void *stream) {
  if (!dY || !dZ16 || !dZT16 || !db || (act && !Z) || M <= 0 || N <= 0) return -1;
  hipLaunchKernelGGL(k_act_backward, dim3(static_cast<unsigned>((M + 63) / 64), static_cast<unsigned>((N + 31) / 32)),
                     dim3(256), 0, static_cast<hipStream_t>(stream), dY, Z, M, N, act, dZ16, dZT16, db);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ugkwp_mlp_adam(float *w, float *m, float *v, const float *g, int64_t n, int64_t cols, float lr, float beta1,
                   float beta2, float eps, int64_t t, uint16_t *w16, uint16_t *wT16, void *stream) {
  if (!w || !m || !v || !g || n <= 0 || cols <= 0 || n % cols || t < 1) return -1;
  const float c1 = 1.0f - powf(beta1, static_cast<float>(t)), c2 = 1.0f - powf(beta2, static_cast<float>(t));
  hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), w, m, v, g, n, cols, lr, beta1, beta2, eps, c1, c2, w16, wT16);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ugkwp_mlp_to_bf16(const float *w, int64_t n, int64_t cols, uint16_t *w16, uint16_t *wT16, void *stream) {
  if (!w || n <= 0 || cols <= 0 || n % cols || (!w16 && !wT16)) return -1;
  hipLaunchKernelGGL(k_to_bf16, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), w, n, cols, w16, wT16);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ugkwp_mlp_pack(const float *W, int64_t out, int64_t in, int32_t permuted, uint16_t *Wf, void *stream) {
  if (!W || !Wf || out <= 0 || in <= 0 || out % 32 || in % 16) return -1;
  const int64_t n = out * in;
  hipLaunchKernelGGL(k_pack_frag, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), W, out, in, permuted ? 1 : 0, Wf);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ugkwp_mlp_forward(const uint16_t *X, int64_t M, int32_t n_layers, const int32_t *widths, const uint16_t *const *Wf,
                      const float *const *bias, float *Y, void *stream) {
  if (!X || !Y || !widths || !Wf || !bias || M <= 0 || M % 32) return -1;
  if (n_layers != 4 || widths[0] != 32 || widths[1] != 256 || widths[2] != 256 || widths[3] != 256 ||
      widths[4] != 32)
    return -1;
  FusedNet net;
  for (int l = 0; l < 4; ++l) {
    if (!Wf[l] || !bias[l]) return -1;
    net.W[l] = Wf[l];
    net.b[l] = bias[l];
  }
  hipLaunchKernelGGL((k_mlp_fused<32, 256, 3, 32>), dim3(static_cast<unsigned>((M / 32 + 3) / 4)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), X, M, net, Y);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ugkwp_mlp_mse_grad(const float *Y, const float *T, int64_t M, int64_t N, int64_t n_out, float scale, float *dY,
                       float *loss, void *stream) {
  if (!Y || !T || !dY || M <= 0 || N <= 0 || n_out <= 0 || n_out > N) return -1;
  const int64_t n = M * N;
  hipLaunchKernelGGL(k_mse_grad, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), Y, T, M, N, n_out, scale, dY, loss);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ugkwp_ws_features(const double *Wc, int32_t nct, int32_t ncr, int32_t nft, int32_t nfr,
                      const ugkwp_ws_case *c, int64_t rows, uint16_t *X16, uint16_t *XT16, float *P32, void *stream) {
  if (!Wc || !X16 || !case_ok(c) || nct < 2 || ncr < 2 || nft < 1 || nfr < 1 ||
      rows < static_cast<int64_t>(nft) * nfr || rows % 32)
    return -1;
  hipLaunchKernelGGL(k_ws_features, dim3(static_cast<unsigned>((rows + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), Wc, nct, ncr, nft, nfr, make_case(c), rows, X16, XT16, P32);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ugkwp_ws_decode(const float *Y, int64_t ldy, const float *P32, int64_t n, const ugkwp_ws_case *c, double *W,
                    void *stream) {
  if (!Y || !P32 || !W || !case_ok(c) || n <= 0 || ldy < 4) return -1;
  hipLaunchKernelGGL(k_ws_decode, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), Y, ldy, P32, n, make_case(c), W);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
