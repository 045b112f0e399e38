// Learned sample budget and finite-source predictor: the perceptron
// 8 -> 128 -> 128 -> 128 -> 2 with erf-GELU activations x Phi(x), whose
// products run on the gfx950 matrix cores in bfloat16 with float32
// accumulation (v_mfma_f32_32x32x16_bf16).  Not part of the paper's method:
// its output only chooses how many limb samples a contour starts with and
// the order in which sources are processed; every magnification is still
// decided by the contour integration's own error estimate.
//
// Parameters live in one float32 vector (the master copy):
//   mean[8], std[8]                   feature standardisation
//   W0 [8 x 128], b0[128]             row-major, input index first
//   W1 [128 x 128], b1, W2 [128 x 128], b2, W3 [128 x 2], b3[2]
// Outputs: out[:, 0] = log2 of the limb-sample count, out[:, 1] = logit of
// "the point-source value misses the tolerance".
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "twk_gelu.h"

namespace twk {
namespace mlp {

constexpr int NF = 8;
constexpr int HID = 128;
constexpr int NO = 2;
constexpr int OFF_MEAN = 0;
constexpr int OFF_STD = 8;
constexpr int OFF_W0 = 16;
constexpr int OFF_B0 = OFF_W0 + NF * HID;
constexpr int OFF_W1 = OFF_B0 + HID;
constexpr int OFF_B1 = OFF_W1 + HID * HID;
constexpr int OFF_W2 = OFF_B1 + HID;
constexpr int OFF_B2 = OFF_W2 + HID * HID;
constexpr int OFF_W3 = OFF_B2 + HID;
constexpr int OFF_B3 = OFF_W3 + HID * NO;
constexpr int NPARAM = OFF_B3 + NO;  // 34450

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Matrix-core operand layout of the 32x32x16 bf16 product (one wave):
//   A (32 x 16): lane l holds A[l % 32][8 (l / 32) + j], j = 0..7
//   B (16 x 32): lane l holds B[8 (l / 32) + j][l % 32]
//   D (32 x 32): lane l, register r holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
__device__ inline int d_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ inline f32x16 mma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// gelu(x) and gelu_grad(x) of the hidden layers: twk_gelu.h

// ---------------------------------------------------------------- packing
// Inference keeps the four weight matrices as ready-made B operands:
// fragment f = (layer block) + ks * NT + nt holds, for each lane, the eight
// bf16 values of k-step ks (16 rows) and n-tile nt (32 columns).
//   layer 0: K = 8 padded to 16 (1 step), 4 n-tiles     -> fragments 0..3
//   layer 1: 8 k-steps x 4 n-tiles                      -> 4..35
//   layer 2: 8 k-steps x 4 n-tiles                      -> 36..67
//   layer 3: 8 k-steps x 1 n-tile (2 columns of 32 used) -> 68..75
constexpr int FRAG_L0 = 0, FRAG_L1 = 4, FRAG_L2 = 36, FRAG_L3 = 68, NFRAG = 76;

__global__ __launch_bounds__(64) void k_pack(const float* __restrict__ P, bf16x8* __restrict__ frag) {
  const int f = blockIdx.x, lane = threadIdx.x;
  int K, N, ks, nt, off;
  if (f < FRAG_L1) { K = NF; N = HID; ks = 0; nt = f; off = OFF_W0; }
  else if (f < FRAG_L2) { K = HID; N = HID; ks = (f - FRAG_L1) / 4; nt = (f - FRAG_L1) % 4; off = OFF_W1; }
  else if (f < FRAG_L3) { K = HID; N = HID; ks = (f - FRAG_L2) / 4; nt = (f - FRAG_L2) % 4; off = OFF_W2; }
  else { K = HID; N = NO; ks = f - FRAG_L3; nt = 0; off = OFF_W3; }
  const int n = 32 * nt + (lane & 31);
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 16 * ks + 8 * (lane >> 5) + j;
    v[j] = (__bf16)((k < K && n < N) ? P[off + k * N + n] : 0.0f);
  }
  frag[f * 64 + lane] = v;
}

// ---------------------------------------------------------------- inference
constexpr int ACT_LD = HID + 8;  // row stride of the activation staging (bf16)
constexpr int INFER_WAVES = 8;  // waves per block sharing one LDS copy of the weights

// Bias, GELU, round to bf16 and stage one 32 x 128 activation tile in LDS.
__device__ inline void stage(__bf16 (*act)[ACT_LD], const f32x16* acc, const float* __restrict__ b,
                             int lane) {
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int c = 32 * nt + (lane & 31);
    const float bc = b[c];
#pragma unroll
    for (int r = 0; r < 16; ++r) act[d_row(lane, r)][c] = (__bf16)gelu(acc[nt][r] + bc);
  }
}

__device__ inline void hidden(__bf16 (*act)[ACT_LD], const bf16x8* __restrict__ W,
                              const float* __restrict__ b, int lane) {
  f32x16 acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[nt][r] = 0.0f;
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) {
    const bf16x8 a = *(const bf16x8*)&act[lane & 31][16 * ks + 8 * (lane >> 5)];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = mma(a, W[(ks * 4 + nt) * 64 + lane], acc[nt]);
  }
  stage(act, acc, b, lane);
}

// One wave per 32-row tile, tiles taken in a grid-stride loop; the packed
// weights sit in LDS for the whole block, activations never leave LDS.
// feat: [n x 8] float32 (raw features); out: [n x 2] float32; the row count
// is n, or *n_dev when given (a device-side count of queued tasks).
// n_long (optional): the rows whose first output is at least long_l2 are
// counted, each as `weight` tasks, into *n_long (one atomic per block), and
// per 32-row tile (rows, unweighted) into tile_long[tile].
__global__ __launch_bounds__(64 * INFER_WAVES) void k_infer(const float* __restrict__ P,
                                                             const bf16x8* __restrict__ frag,
                                                             int64_t n, const long long* __restrict__ n_dev,
                                                             const float* __restrict__ feat,
                                                             float* __restrict__ out,
                                                             long long* __restrict__ n_long,
                                                             float long_l2, int weight,
                                                             int32_t* __restrict__ tile_long) {
  __shared__ bf16x8 w[NFRAG * 64];
  __shared__ __bf16 act[INFER_WAVES][32][ACT_LD];
  __shared__ float pb[3 * HID + NO + 2 * NF];
  __shared__ unsigned block_long;
  if (threadIdx.x == 0) block_long = 0u;
  for (int i = threadIdx.x; i < NFRAG * 64; i += blockDim.x) w[i] = frag[i];
  for (int i = threadIdx.x; i < HID; i += blockDim.x) {
    pb[i] = P[OFF_B0 + i];
    pb[HID + i] = P[OFF_B1 + i];
    pb[2 * HID + i] = P[OFF_B2 + i];
  }
  if (threadIdx.x < NO) pb[3 * HID + threadIdx.x] = P[OFF_B3 + threadIdx.x];
  if (threadIdx.x < 2 * NF) pb[3 * HID + NO + threadIdx.x] = P[threadIdx.x];
  __syncthreads();
  if (n_dev) n = *n_dev;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float* mean = &pb[3 * HID + NO];
  const float* sd = mean + NF;
  const int64_t ntile = (n + 31) / 32;
  unsigned nl = 0u;
  for (int64_t t = (int64_t)blockIdx.x * INFER_WAVES + wave; t < ntile;
       t += (int64_t)gridDim.x * INFER_WAVES) {
    const int64_t r0 = t * 32;
    bf16x8 a;
    {
      const int64_t row = r0 + (lane & 31);
      const bool on = lane < 32 && row < n;
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] = (__bf16)(on ? (feat[row * NF + j] - mean[j]) / sd[j] : 0.0f);
    }
    f32x16 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[nt][r] = 0.0f;
      acc[nt] = mma(a, w[(FRAG_L0 + nt) * 64 + lane], acc[nt]);
    }
    stage(act[wave], acc, &pb[0], lane);
    hidden(act[wave], &w[FRAG_L1 * 64], &pb[HID], lane);
    hidden(act[wave], &w[FRAG_L2 * 64], &pb[2 * HID], lane);
    f32x16 o;
#pragma unroll
    for (int r = 0; r < 16; ++r) o[r] = 0.0f;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const bf16x8 x = *(const bf16x8*)&act[wave][lane & 31][16 * ks + 8 * (lane >> 5)];
      o = mma(x, w[(FRAG_L3 + ks) * 64 + lane], o);
    }
    const int col = lane & 31;
    unsigned tl = 0u;
    if (col < NO) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = r0 + d_row(lane, r);
        if (row < n) {
          const float v = o[r] + pb[3 * HID + col];
          out[row * NO + col] = v;
          tl += (col == 0 && v >= long_l2) ? 1u : 0u;
        }
      }
    }
    nl += tl;
    if (tile_long) {
      tl += __shfl_down(tl, 32);
      if (lane == 0) tile_long[t] = (int32_t)tl;
    }
  }
  if (n_long) {
    if (nl) atomicAdd(&block_long, nl);
    __syncthreads();
    if (threadIdx.x == 0 && block_long)
      atomicAdd((unsigned long long*)n_long, (unsigned long long)block_long * (unsigned)weight);
  }
}

// ---------------------------------------------------------------- training
// C (+)= A B with A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn],
// operands float32 in memory, rounded to bf16 at the load; one wave per
// 32 x 32 tile of C; blockIdx.z splits K, each split writing its partial
// product to work[z][M][N] for a deterministic sum afterwards.
struct Gemm {
  const float* A;
  int64_t sam, sak;
  const float* B;
  int64_t sbk, sbn;
  float* C;
  int64_t scm, scn;
  int M, N, K, ksplit;
  float* work;
};

__global__ __launch_bounds__(64) void k_gemm(Gemm g) {
  const int lane = threadIdx.x;
  const int m0 = blockIdx.x * 32, n0 = blockIdx.y * 32, z = blockIdx.z;
  const int kc = ((g.K + 16 * g.ksplit - 1) / (16 * g.ksplit)) * 16;
  const int kb = z * kc, ke = min(g.K, kb + kc);
  const int mi = m0 + (lane & 31), nj = n0 + (lane & 31);
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int k0 = kb; k0 < ke; k0 += 16) {
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + 8 * (lane >> 5) + j;
      const bool kin = k < ke;
      a[j] = (__bf16)((kin && mi < g.M) ? g.A[(int64_t)mi * g.sam + (int64_t)k * g.sak] : 0.0f);
      b[j] = (__bf16)((kin && nj < g.N) ? g.B[(int64_t)k * g.sbk + (int64_t)nj * g.sbn] : 0.0f);
    }
    acc = mma(a, b, acc);
  }
  if (nj >= g.N) return;
  if (g.ksplit > 1) {
    float* dst = g.work + (int64_t)z * g.M * g.N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = m0 + d_row(lane, r);
      if (i < g.M) dst[(int64_t)i * g.N + nj] = acc[r];
    }
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = m0 + d_row(lane, r);
      if (i < g.M) g.C[(int64_t)i * g.scm + (int64_t)nj * g.scn] = acc[r];
    }
  }
}

__global__ void k_split_sum(const float* __restrict__ work, int ksplit, int M, int N, float* C,
                            int64_t scm, int64_t scn) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  float s = 0.0f;
  for (int z = 0; z < ksplit; ++z) s += work[(int64_t)z * M * N + i];
  C[(i / N) * scm + (i % N) * scn] = s;
}

// Z += b (row broadcast); H = gelu(Z) when H is given.
__global__ void k_bias_act(float* Z, const float* __restrict__ b, float* H, int64_t rows, int N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * N) return;
  const float z = Z[i] + b[i % N];
  Z[i] = z;
  if (H) H[i] = gelu(z);
}

// dZ = dH * gelu'(Z), in place on dH.
__global__ void k_gelu_bwd(float* dH, const float* __restrict__ Z, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dH[i] *= gelu_grad(Z[i]);
}

// Mean Huber on out[:,0] and mean BCE-with-logits on out[:,1]; gradient of
// the mean loss into dO, per-row loss into lrow.
__global__ void k_loss(const float* __restrict__ O, const float* __restrict__ yb,
                       const float* __restrict__ yf, float delta, int64_t rows, float* dO,
                       float* lrow) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const float r = O[2 * i] - yb[i];
  const float ar = fabsf(r);
  const float hub = ar <= delta ? 0.5f * r * r : delta * (ar - 0.5f * delta);
  const float o = O[2 * i + 1], y = yf[i];
  const float bce = fmaxf(o, 0.0f) - o * y + log1pf(expf(-fabsf(o)));
  const float inv = 1.0f / (float)rows;
  dO[2 * i] = fminf(fmaxf(r, -delta), delta) * inv;
  dO[2 * i + 1] = (1.0f / (1.0f + expf(-o)) - y) * inv;
  lrow[i] = hub + bce;
}

// Column sums of a [rows x N] matrix (one thread per column, fixed order).
__global__ void k_colsum(const float* __restrict__ X, int64_t rows, int N, float* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  float s = 0.0f;
  for (int64_t r = 0; r < rows; ++r) s += X[r * N + c];
  out[c] = s;
}

// Deterministic sum of n floats into one double (single block).
__global__ __launch_bounds__(256) void k_sum(const float* __restrict__ x, int64_t n, double* out) {
  __shared__ double part[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

// Gather a minibatch through a permutation and standardise its features.
__global__ void k_gather(const float* __restrict__ feat, const float* __restrict__ yb,
                         const float* __restrict__ yf, const int32_t* __restrict__ idx,
                         int64_t rows, const float* __restrict__ P, float* X, float* byb,
                         float* byf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const int64_t s = idx ? idx[i] : i;
#pragma unroll
  for (int j = 0; j < NF; ++j) X[i * NF + j] = (feat[s * NF + j] - P[OFF_MEAN + j]) / P[OFF_STD + j];
  byb[i] = yb[s];
  byf[i] = yf[s];
}

// Adam with bias correction on the trainable part of the parameter vector.
__global__ void k_adam(float* P, const float* __restrict__ G, float* m, float* v, int64_t n0,
                       int64_t n1, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = n0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n1) return;
  const float g = G[i];
  const float mi = b1 * m[i] + (1.0f - b1) * g;
  const float vi = b2 * v[i] + (1.0f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Per-block partial sums and sums of squares of the eight features, in
// double; the host adds the blocks in order.
__global__ __launch_bounds__(256) void k_feat_stats(const float* __restrict__ feat, int64_t n,
                                                    double* part) {
  __shared__ double acc[256][2 * NF];
  double s[2 * NF];
#pragma unroll
  for (int j = 0; j < 2 * NF; ++j) s[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      const double x = feat[i * NF + j];
      s[j] += x;
      s[NF + j] += x * x;
    }
  }
#pragma unroll
  for (int j = 0; j < 2 * NF; ++j) acc[threadIdx.x][j] = s[j];
  __syncthreads();
  if (threadIdx.x < 2 * NF) {
    double t = 0.0;
    for (int k = 0; k < 256; ++k) t += acc[k][threadIdx.x];
    part[blockIdx.x * 2 * NF + threadIdx.x] = t;
  }
}

}  // namespace mlp
}  // namespace twk
