// Learned spectral preconditioner of the damped step (an extension of
// Eq. dampstep: the paper's damping x0 / (E0 + T_k) is fixed).
//
// The plain step is phi = psi - x0 F^-1[F r / (E0 + T_k)], r = h psi - <h> psi.
// The learned step multiplies the damping, per state alpha and |k| shell s,
// by a gain g = GMAX sigmoid(o), o = MLP(features(alpha, s)):
//   x0 = |k| at the shell centre / |k|max,   x1 = <h>_alpha / E0,
//   x2 = log10(P_s / P + 1e-12) / 6 + 1   (share of the residual's spectral
//        power in shell s),                 x3 = T_k at the shell centre / E0.
// The MLP is 4 -> 128 -> 128 -> 128 -> 1 with ReLU, BF16 weights (rounded
// from FP32 master weights, round to nearest even) and FP32 accumulation.
//
// Training targets come from the solver's own iterates.  For a sampled state,
// the step restricted to shell s is d_s = x0 F^-1[1_s F r / (E0 + T_k)]; to
// first order, with the mean field frozen, the residual after the step
// psi - sum_s g_s d_s is r - sum_s g_s w_s with w_s = (h - <h>) d_s, and the
// target gains minimise |r - sum_s g_s w_s|^2 (real g, normal equations with
// a small ridge, clamped to [0, GMAX]).  The loss is the residual-power
// weighted mean square error of the gains; training is Adam on the GPU with
// this file's forward and backward kernels.
#include <cmath>
#include <random>
#include <vector>

#include "sky_kernels.h"

namespace sky {

namespace {
constexpr int PIN = 4;
constexpr int PH = 128;
constexpr float GMAX = 4.0f;
// parameter offsets: W1[PH][PIN], b1[PH], W2[PH][PH], b2, W3[PH][PH], b3, W4[PH], b4
constexpr int OW1 = 0, OB1 = OW1 + PH * PIN, OW2 = OB1 + PH, OB2 = OW2 + PH * PH,
              OW3 = OB2 + PH, OB3 = OW3 + PH * PH, OW4 = OB3 + PH, OB4 = OW4 + PH,
              NPAR = OB4 + 1;
constexpr int NS_MAX = 32;   // sampled states per collection

__device__ inline float bf16_round(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__global__ void k_round_params(const float* __restrict__ p, float* __restrict__ q, int n, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = bf16_round(p[i]);
}

// ---- forward pass on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16)
// One wave carries 16 samples through the MLP.  The two 128 x 128 layers are
// MFMA products: the weights are BF16 values already (the parameters are
// rounded by k_round_params), and each FP32 activation is split exactly into
// three BF16 terms h = t0 + t1 + t2 (8 significant bits each, rounded to
// nearest at each step), so that every product t_i w is exact in FP32 and
// the layer is FP32 activations x BF16 weights with FP32 accumulation, as
// the scalar form, up to the order of the sums.  MFMA operands: lane l
// supplies 8 consecutive contraction elements starting at 8 (l / 16) of row
// (A: sample) or column (B: neuron) l % 16; register e of lane l returns
// sample 4 (l / 16) + e, neuron l % 16.  The first (4 inputs) and last
// (1 output) layers are scalar.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int FR = 16;         // samples per wave
constexpr int FWV = 4;         // waves per workgroup
constexpr int FLP = PH + 4;    // LDS row pitch of the activations (floats)

__device__ inline unsigned short bf16_hi(float x) { return (unsigned short)(__float_as_uint(x) >> 16); }

// 128 -> 128 layer of one wave: out = relu(bias + in W^T), in and out in LDS
// ([FR][FLP]); W row-major [PH][PH] (BF16 values).
__device__ inline void mlp_layer_mfma(const float* in, float* out, const float* __restrict__ W,
                                      const float* __restrict__ bias, int lane) {
  const int r = lane & 15, kg = (lane >> 4) * 8;
  us8 a[PH / 32][3];
#pragma unroll
  for (int ks = 0; ks < PH / 32; ++ks)
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const float x = in[r * FLP + ks * 32 + kg + t];
      const float x0 = bf16_round(x), x1 = bf16_round(x - x0), x2 = bf16_round(x - x0 - x1);
      a[ks][0][t] = bf16_hi(x0);
      a[ks][1][t] = bf16_hi(x1);
      a[ks][2][t] = bf16_hi(x2);
    }
#pragma unroll
  for (int j = 0; j < PH / 16; ++j) {
    const int n = j * 16 + r;
    f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < PH / 32; ++ks) {
      const float4* wp = reinterpret_cast<const float4*>(W + n * PH + ks * 32 + kg);
      const float4 w0 = wp[0], w1 = wp[1];
      const us8 wb = {bf16_hi(w0.x), bf16_hi(w0.y), bf16_hi(w0.z), bf16_hi(w0.w),
                      bf16_hi(w1.x), bf16_hi(w1.y), bf16_hi(w1.z), bf16_hi(w1.w)};
      const bf8 b = __builtin_bit_cast(bf8, wb);
#pragma unroll
      for (int t = 0; t < 3; ++t)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a[ks][t]), b, acc, 0, 0, 0);
    }
    const float bn = bias[n];
#pragma unroll
    for (int e = 0; e < 4; ++e) out[(4 * (lane >> 4) + e) * FLP + n] = fmaxf(acc[e] + bn, 0.0f);
  }
}

// Forward pass of FR samples per wave, FWV waves per workgroup.  H1..H3 (may
// be null) keep the activations for the backward pass; O the outputs.
__global__ void __launch_bounds__(64 * FWV)
k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ X, int ldx, int B,
          float* __restrict__ H1, float* __restrict__ H2, float* __restrict__ H3,
          float* __restrict__ O, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ float hs[FWV][2][FR * FLP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int b0 = (blockIdx.x * FWV + wv) * FR;
  float* ha = hs[wv][0];
  float* hb = hs[wv][1];
  // layer 1: lane -> neurons lane, lane + 64
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int n = lane + 64 * q;
    float w1[PIN];
#pragma unroll
    for (int i = 0; i < PIN; ++i) w1[i] = P[OW1 + n * PIN + i];
    const float bn = P[OB1 + n];
    for (int s = 0; s < FR; ++s) {
      float a = bn;
      if (b0 + s < B)
#pragma unroll
        for (int i = 0; i < PIN; ++i) a += w1[i] * X[size_t(b0 + s) * ldx + i];
      ha[s * FLP + n] = fmaxf(a, 0.0f);
    }
  }
  __syncthreads();
  mlp_layer_mfma(ha, hb, P + OW2, P + OB2, lane);
  __syncthreads();
  if (H1)
    for (int s = 0; s < FR; ++s)
      if (b0 + s < B) {
        H1[size_t(b0 + s) * PH + lane] = ha[s * FLP + lane];
        H1[size_t(b0 + s) * PH + lane + 64] = ha[s * FLP + lane + 64];
      }
  __syncthreads();
  mlp_layer_mfma(hb, ha, P + OW3, P + OB3, lane);
  __syncthreads();
  if (H2 || H3)
    for (int s = 0; s < FR; ++s)
      if (b0 + s < B)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int n = lane + 64 * q;
          if (H2) H2[size_t(b0 + s) * PH + n] = hb[s * FLP + n];
          if (H3) H3[size_t(b0 + s) * PH + n] = ha[s * FLP + n];
        }
  // layer 4: sample lane % 16, a quarter of the neurons per lane, then the
  // four quarters summed in a fixed order
  const int s = lane & 15, k0 = (lane >> 4) * (PH / 4);
  float v = 0.0f;
  for (int k = 0; k < PH / 4; ++k) v += P[OW4 + k0 + k] * ha[s * FLP + k0 + k];
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  if (lane < FR && b0 + s < B) O[b0 + s] = v + P[OB4];
}

// dL/do per sample and the loss terms: g = GMAX sigmoid(o),
// L = sum_b w_b (g_b - t_b)^2 / sum_b w_b.  S = [x0..x3, t, w] rows.
__global__ void k_mlp_loss(const float* __restrict__ O, const float* __restrict__ S, int B,
                           double wsum, float* __restrict__ dO, double* __restrict__ lpart, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (b < B) {
    const float t = S[size_t(b) * 6 + 4], w = S[size_t(b) * 6 + 5];
    const float sg = 1.0f / (1.0f + expf(-O[b]));
    const float g = GMAX * sg;
    const float e = g - t;
    l = double(w) * double(e) * double(e) / wsum;
    dO[b] = float(2.0 * double(w) * double(e) / wsum) * GMAX * sg * (1.0f - sg);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// One backward layer of one wave on the BF16 matrix cores: out[s][j] =
// relu'(Hp[b0 + s][j]) sum_i in[s][i] W[i][j] (W row-major [PH][PH], BF16
// values), also stored to Dout for the weight gradients.  Operands and
// splits as in mlp_layer_mfma, with W's columns as the B operand.
__device__ inline void mlp_layer_bwd_mfma(const float* in, float* out, const float* __restrict__ W,
                                          const float* __restrict__ Hp, float* __restrict__ Dout,
                                          int b0, int B, int lane) {
  const int r = lane & 15, kg = (lane >> 4) * 8;
  us8 a[PH / 32][3];
#pragma unroll
  for (int ks = 0; ks < PH / 32; ++ks)
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const float x = in[r * FLP + ks * 32 + kg + t];
      const float x0 = bf16_round(x), x1 = bf16_round(x - x0), x2 = bf16_round(x - x0 - x1);
      a[ks][0][t] = bf16_hi(x0);
      a[ks][1][t] = bf16_hi(x1);
      a[ks][2][t] = bf16_hi(x2);
    }
#pragma unroll
  for (int jb = 0; jb < PH / 16; ++jb) {
    const int j = jb * 16 + r;
    f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < PH / 32; ++ks) {
      us8 wb;
#pragma unroll
      for (int t = 0; t < 8; ++t) wb[t] = bf16_hi(W[(ks * 32 + kg + t) * PH + j]);
      const bf8 b = __builtin_bit_cast(bf8, wb);
#pragma unroll
      for (int t = 0; t < 3; ++t)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a[ks][t]), b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int sr = 4 * (lane >> 4) + e, b = b0 + sr;
      float v = 0.0f;
      if (b < B) {
        v = Hp[size_t(b) * PH + j] > 0.0f ? acc[e] : 0.0f;
        Dout[size_t(b) * PH + j] = v;
      }
      out[sr * FLP + j] = v;
    }
  }
}

// dL/d(pre-activation) of the three hidden layers, FR samples per wave:
// D3 = dO W4 relu'(H3), D2 = (D3 W3) relu'(H2), D1 = (D2 W2) relu'(H1).
__global__ void __launch_bounds__(64 * FWV)
k_mlp_bwd_act(const float* __restrict__ P, const float* __restrict__ H1,
              const float* __restrict__ H2, const float* __restrict__ H3,
              const float* __restrict__ dO, int B, float* __restrict__ D1,
              float* __restrict__ D2, float* __restrict__ D3, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ float hs[FWV][2][FR * FLP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int b0 = (blockIdx.x * FWV + wv) * FR;
  float* da = hs[wv][0];
  float* db = hs[wv][1];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int n = lane + 64 * q;
    const float w4 = P[OW4 + n];
    for (int sr = 0; sr < FR; ++sr) {
      const int b = b0 + sr;
      float v = 0.0f;
      if (b < B) {
        v = H3[size_t(b) * PH + n] > 0.0f ? dO[b] * w4 : 0.0f;
        D3[size_t(b) * PH + n] = v;
      }
      da[sr * FLP + n] = v;
    }
  }
  __syncthreads();
  mlp_layer_bwd_mfma(da, db, P + OW3, H2, D2, b0, B, lane);
  __syncthreads();
  mlp_layer_bwd_mfma(db, da, P + OW2, H1, D1, b0, B, lane);
}

// ---- parameter gradient
// x = v[0][t] + v[1][t] + v[2][t] as three BF16 bit patterns (exact for
// normal FP32 x: 8 significant bits per term, rounded to nearest at each step).
__device__ inline void split3_at(float x, us8 (&v)[3], int t) {
  const float a = bf16_round(x), b = bf16_round(x - a), c = bf16_round(x - a - b);
  v[0][t] = bf16_hi(a);
  v[1][t] = bf16_hi(b);
  v[2][t] = bf16_hi(c);
}

constexpr int GCH = 64;    // samples per chunk of the gradient partials
constexpr int GSUB = 32;   // samples per MFMA step (the contraction of one MFMA)

// Partial gradient of every parameter over the samples of chunk blockIdx.x:
// part[chunk][p].  The two 128 x 128 weight blocks are D^T H over the chunk
// on the BF16 matrix cores: both FP32 operands split in three BF16 terms,
// the six products t_i u_j with i + j <= 2 (the dropped ones are below
// 2^-24 of the product), FP32 accumulation; wave w owns the output rows
// 32 w .. 32 w + 31 of both blocks.  W1, the biases, W4 and b4 are FP32
// sums over the chunk, one thread per parameter.  The chunk goes through LDS
// GSUB samples at a time.
__global__ void __launch_bounds__(256)
k_mlp_grad_part(const float* __restrict__ S, const float* __restrict__ H1,
                const float* __restrict__ H2, const float* __restrict__ H3,
                const float* __restrict__ dO, const float* __restrict__ D1,
                const float* __restrict__ D2, const float* __restrict__ D3, int B,
                float* __restrict__ part, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ float ds[2][GSUB][FLP], hs[2][GSUB][FLP];   // (D2, H1), (D3, H2)
  __shared__ float d1s[GSUB][FLP], h3s[GSUB][FLP], xs[GSUB][PIN], dos[GSUB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c0 = blockIdx.x * GCH, c1 = min(B, c0 + GCH);
  float* out = part + size_t(blockIdx.x) * NPAR;
  const int r = lane & 15, kg = (lane >> 4) * 8;
  f4v acc[2][2][PH / 16];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int ib = 0; ib < PH / 16; ++ib) acc[m][jb][ib] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
  constexpr int PI[6] = {0, 0, 1, 0, 1, 2};
  constexpr int PJ[6] = {0, 1, 0, 2, 1, 0};
  // W1, b1, b2, b3, W4, b4: thread tid owns parameters tid + 256 q
  constexpr int NSMALL = PH * PIN + 4 * PH + 1;
  constexpr int NQ = (NSMALL + 255) / 256;
  float sv[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) sv[q] = 0.0f;
  for (int s0 = c0; s0 < c1; s0 += GSUB) {
    __syncthreads();
    for (int e = tid; e < GSUB * PH; e += 256) {
      const int sr = e / PH, n = e % PH, b = s0 + sr;
      const bool ok = b < c1;
      const size_t o = size_t(b) * PH + n;
      ds[0][sr][n] = ok ? D2[o] : 0.0f;
      hs[0][sr][n] = ok ? H1[o] : 0.0f;
      ds[1][sr][n] = ok ? D3[o] : 0.0f;
      hs[1][sr][n] = ok ? H2[o] : 0.0f;
      d1s[sr][n] = ok ? D1[o] : 0.0f;
      h3s[sr][n] = ok ? H3[o] : 0.0f;
    }
    if (tid < GSUB * PIN) {
      const int sr = tid / PIN, i = tid % PIN, b = s0 + sr;
      xs[sr][i] = b < c1 ? S[size_t(b) * 6 + i] : 0.0f;
    }
    if (tid < GSUB) dos[tid] = s0 + tid < c1 ? dO[s0 + tid] : 0.0f;
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      us8 a[2][3];
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int t = 0; t < 8; ++t) split3_at(ds[m][kg + t][(2 * wv + jb) * 16 + r], a[jb], t);
#pragma unroll
      for (int ib = 0; ib < PH / 16; ++ib) {
        us8 u[3];
#pragma unroll
        for (int t = 0; t < 8; ++t) split3_at(hs[m][kg + t][ib * 16 + r], u, t);
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
          for (int q = 0; q < 6; ++q)
            acc[m][jb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf8, a[jb][PI[q]]), __builtin_bit_cast(bf8, u[PJ[q]]),
                acc[m][jb][ib], 0, 0, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int p = tid + 256 * q;
      float v = 0.0f;
      if (p < PH * PIN) {                          // W1[j][i]: D1[b][j] x[b][i]
        const int j = p / PIN, i = p % PIN;
        for (int sr = 0; sr < GSUB; ++sr) v += d1s[sr][j] * xs[sr][i];
      } else if (p < PH * PIN + 3 * PH) {          // b1, b2, b3
        const int l = (p - PH * PIN) / PH, j = (p - PH * PIN) % PH;
        for (int sr = 0; sr < GSUB; ++sr) v += l == 0 ? d1s[sr][j] : ds[l - 1][sr][j];
      } else if (p < PH * PIN + 4 * PH) {          // W4[i]: dO[b] H3[b][i]
        const int i = p - PH * PIN - 3 * PH;
        for (int sr = 0; sr < GSUB; ++sr) v += dos[sr] * h3s[sr][i];
      } else if (p < NSMALL) {                     // b4
        for (int sr = 0; sr < GSUB; ++sr) v += dos[sr];
      }
      sv[q] += v;
    }
  }
  // output rows j (neuron of the layer's output) and columns i (its input)
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int ib = 0; ib < PH / 16; ++ib)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = (2 * wv + jb) * 16 + 4 * (lane >> 4) + e, i = ib * 16 + r;
          out[(m ? OW3 : OW2) + j * PH + i] = acc[m][jb][ib][e];
        }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int p = tid + 256 * q;
    if (p < PH * PIN) out[OW1 + p] = sv[q];
    else if (p < PH * PIN + 3 * PH) {
      const int l = (p - PH * PIN) / PH, j = (p - PH * PIN) % PH;
      out[(l == 0 ? OB1 : l == 1 ? OB2 : OB3) + j] = sv[q];
    } else if (p < PH * PIN + 4 * PH) out[OW4 + p - PH * PIN - 3 * PH] = sv[q];
    else if (p < NSMALL) out[OB4] = sv[q];
  }
}

// G[p] = sum over the chunks of part[chunk][p], in chunk order.
__global__ void k_mlp_grad_sum(const float* __restrict__ part, int nchunk, float* __restrict__ G,
                               const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAR) return;
  float v = 0.0f;
#pragma unroll 8
  for (int c = 0; c < nchunk; ++c) v += part[size_t(c) * NPAR + p];
  G[p] = v;
}

__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                       float* __restrict__ V, int n, float lr, float b1, float b2, float c1,
                       float c2, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float m = b1 * M[i] + (1.0f - b1) * g;
  const float v = b2 * V[i] + (1.0f - b2) * g * g;
  M[i] = m;
  V[i] = v;
  P[i] -= lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
}

__global__ void k_sum_d(const double* __restrict__ part, int n, double* __restrict__ out, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  if (threadIdx.x) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  out[0] = s;
}

// Features of (state alpha, shell s) rows: X[(a*S + s)][0..3] (row length 6).
__global__ void k_pc_features(const double* __restrict__ pow, const double* __restrict__ eps,
                              int stride, int ns, double e0, double hb2m, double kmax,
                              float* __restrict__ X, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ns * PC_SHELLS) return;
  const int a = r / PC_SHELLS, s = r % PC_SHELLS;
  const int al = a * stride;
  double ptot = 0.0;
  for (int t = 0; t < PC_SHELLS; ++t) ptot += pow[size_t(al) * PC_SHELLS + t];
  const double frac = ptot > 0.0 ? pow[size_t(al) * PC_SHELLS + s] / ptot : 0.0;
  const double kc = (s + 0.5) / PC_SHELLS;
  float* x = X + size_t(r) * 6;
  x[0] = float(kc);
  x[1] = float(eps[al] / e0);
  x[2] = float(log10(frac + 1e-12) / 6.0 + 1.0);
  x[3] = float(hb2m * (kc * kmax) * (kc * kmax) / e0);
  x[5] = float(frac);   // sample weight: share of the residual in the shell
}

// gain[r] = GMAX sigmoid(O[r])
__global__ void k_pc_gains(const float* __restrict__ O, int n, float* __restrict__ gain, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) gain[r] = GMAX / (1.0f + expf(-O[r]));
}

// Batch b = a*S + s of the sampled states: copies of psi, h psi, <h> and a
// one-hot gain row selecting shell s.
template <typename T>
__global__ void k_pc_gather(const T* __restrict__ psi, const T* __restrict__ hpsi,
                            const double* __restrict__ eps, const int* __restrict__ idx,
                            long V, T* __restrict__ bpsi, T* __restrict__ bh,
                            double* __restrict__ beps, float* __restrict__ onehot, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int b = blockIdx.y, a = b / PC_SHELLS, s = b % PC_SHELLS;
  const size_t src = size_t(idx[a]) * V, dst = size_t(b) * V;
  for (long e = long(blockIdx.x) * blockDim.x + threadIdx.x; e < V; e += long(gridDim.x) * blockDim.x) {
    bpsi[dst + e] = psi[src + e];
    bh[dst + e] = hpsi[src + e];
  }
  if (blockIdx.x == 0 && threadIdx.x < PC_SHELLS) {
    onehot[size_t(b) * PC_SHELLS + threadIdx.x] = threadIdx.x == s ? 1.0f : 0.0f;
    if (threadIdx.x == 0) beps[b] = eps[idx[a]];
  }
}

// d = psi - phi (in place in phi)
template <typename T>
__global__ void k_pc_dir(const T* __restrict__ bpsi, T* __restrict__ bphi, size_t n, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < n) {
    const T a = bpsi[e];
    T b = bphi[e];
    b.x = a.x - b.x;
    b.y = a.y - b.y;
    bphi[e] = b;
  }
}

// Gram partials per sampled state: w_s = h d_s - eps d_s, r = h psi - eps psi;
// part[a][blk][q] for q < S(S+1)/2 (s <= t) then S entries <w_s, r>.
constexpr int NG = PC_SHELLS * (PC_SHELLS + 1) / 2 + PC_SHELLS;
template <typename T>
__global__ void __launch_bounds__(256)
k_pc_gram(const T* __restrict__ bpsi, const T* __restrict__ bh, const T* __restrict__ bd,
          const T* __restrict__ bhd, const double* __restrict__ beps, long V,
          double* __restrict__ part, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int a = blockIdx.y;
  double acc[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) acc[q] = 0.0;
  const size_t b0 = size_t(a) * PC_SHELLS;
  const double e = beps[b0];
  for (long x = long(blockIdx.x) * blockDim.x + threadIdx.x; x < V; x += long(gridDim.x) * blockDim.x) {
    double wr[PC_SHELLS], wi[PC_SHELLS];
#pragma unroll
    for (int s = 0; s < PC_SHELLS; ++s) {
      const T d = bd[(b0 + s) * V + x], hd = bhd[(b0 + s) * V + x];
      wr[s] = double(hd.x) - e * double(d.x);
      wi[s] = double(hd.y) - e * double(d.y);
    }
    const T p = bpsi[b0 * V + x], h = bh[b0 * V + x];
    const double rr = double(h.x) - e * double(p.x), ri = double(h.y) - e * double(p.y);
    int q = 0;
#pragma unroll
    for (int s = 0; s < PC_SHELLS; ++s)
#pragma unroll
      for (int t = s; t < PC_SHELLS; ++t) acc[q++] += wr[s] * wr[t] + wi[s] * wi[t];
#pragma unroll
    for (int s = 0; s < PC_SHELLS; ++s) acc[q++] += wr[s] * rr + wi[s] * ri;
  }
  __shared__ double red[4][NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    double v = acc[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < NG)
    part[(size_t(a) * gridDim.x + blockIdx.x) * NG + threadIdx.x] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// Per sampled state: sum the Gram partials, solve (G + lam 1) g = c by
// Cholesky (FP64), clamp to [0, GMAX], write the target column t of the
// sample rows.  One thread per state.
__global__ void k_pc_solve(const double* __restrict__ part, int nblk, int ns, float* __restrict__ S, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= ns) return;
  double Gm[PC_SHELLS][PC_SHELLS], c[PC_SHELLS];
  double sum[NG];
  for (int q = 0; q < NG; ++q) sum[q] = 0.0;
  for (int k = 0; k < nblk; ++k)
    for (int q = 0; q < NG; ++q) sum[q] += part[(size_t(a) * nblk + k) * NG + q];
  int q = 0;
  for (int s = 0; s < PC_SHELLS; ++s)
    for (int t = s; t < PC_SHELLS; ++t) { Gm[s][t] = sum[q]; Gm[t][s] = sum[q]; ++q; }
  for (int s = 0; s < PC_SHELLS; ++s) c[s] = sum[q++];
  double tr = 0.0;
  for (int s = 0; s < PC_SHELLS; ++s) tr += Gm[s][s];
  const double lam = 1e-6 * tr / PC_SHELLS + 1e-300;
  for (int s = 0; s < PC_SHELLS; ++s) Gm[s][s] += lam;
  // Cholesky in place (lower)
  for (int k = 0; k < PC_SHELLS; ++k) {
    double d = Gm[k][k];
    for (int l = 0; l < k; ++l) d -= Gm[k][l] * Gm[k][l];
    d = sqrt(fmax(d, 1e-300));
    Gm[k][k] = d;
    for (int i = k + 1; i < PC_SHELLS; ++i) {
      double v = Gm[i][k];
      for (int l = 0; l < k; ++l) v -= Gm[i][l] * Gm[k][l];
      Gm[i][k] = v / d;
    }
  }
  double y[PC_SHELLS], g[PC_SHELLS];
  for (int i = 0; i < PC_SHELLS; ++i) {
    double v = c[i];
    for (int l = 0; l < i; ++l) v -= Gm[i][l] * y[l];
    y[i] = v / Gm[i][i];
  }
  for (int i = PC_SHELLS - 1; i >= 0; --i) {
    double v = y[i];
    for (int l = i + 1; l < PC_SHELLS; ++l) v -= Gm[l][i] * g[l];
    g[i] = v / Gm[i][i];
  }
  for (int s = 0; s < PC_SHELLS; ++s)
    S[(size_t(a) * PC_SHELLS + s) * 6 + 4] = float(fmin(fmax(g[s], 0.0), double(GMAX)));
}
}  // namespace

int precond_nparams() { return NPAR; }
int precond_ns_max() { return NS_MAX; }

void precond_init_params(float* P_dev, unsigned seed, hipStream_t st) {
  std::vector<float> h(NPAR, 0.0f);
  std::mt19937 rng(seed);
  auto fill = [&](int off, int fan_in, int fan_out) {
    const float a = std::sqrt(6.0f / float(fan_in + fan_out));
    std::uniform_real_distribution<float> u(-a, a);
    for (int i = 0; i < fan_in * fan_out; ++i) h[off + i] = u(rng);
  };
  fill(OW1, PIN, PH);
  fill(OW2, PH, PH);
  fill(OW3, PH, PH);
  fill(OW4, PH, 1);
  for (int j = 0; j < PH; ++j) { h[OB1 + j] = 0.01f; h[OB2 + j] = 0.01f; h[OB3 + j] = 0.01f; }
  for (int j = 0; j < PH; ++j) h[OW4 + j] *= 0.1f;
  h[OB4] = std::log(1.0f / (GMAX - 1.0f));   // gain 1 at the start: the plain damping
  hipMemcpyAsync(P_dev, h.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice, st);
  hipStreamSynchronize(st);
}

void precond_round(const float* P, float* Pb, hipStream_t st) {
  hipLaunchKernelGGL(k_round_params, dim3((NPAR + 255) / 256), dim3(256), 0, st, P, Pb, NPAR, g_launch_gate);
}

void precond_forward(const float* Pb, const float* X, int B, float* H1, float* H2, float* H3,
                     float* O, hipStream_t st) {
  if (B <= 0) return;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((B + FR * FWV - 1) / (FR * FWV)), dim3(64 * FWV), 0, st, Pb, X,
                     6, B, H1, H2, H3, O, g_launch_gate);
}

void precond_features(const double* pow, const double* eps, int stride, int ns, double e0,
                      double hb2m, double kmax, float* X, hipStream_t st) {
  const int n = ns * PC_SHELLS;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pc_features, dim3((n + 127) / 128), dim3(128), 0, st, pow, eps, stride, ns,
                     e0, hb2m, kmax, X, g_launch_gate);
}

void precond_gains(const float* O, int n, float* gain, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pc_gains, dim3((n + 255) / 256), dim3(256), 0, st, O, n, gain, g_launch_gate);
}

double precond_loss_grad(const float* Pb, const float* S, int B, double wsum, float* H1,
                         float* H2, float* H3, float* O, float* dO, float* D1, float* D2,
                         float* D3, float* G, float* gpart, double* dscratch, int want_loss,
                         hipStream_t st) {
  if (B <= 0) return 0.0;
  precond_forward(Pb, S, B, H1, H2, H3, O, st);
  const int nb = (B + 255) / 256;
  hipLaunchKernelGGL(k_mlp_loss, dim3(nb), dim3(256), 0, st, (const float*)O, S, B, wsum, dO,
                     dscratch, g_launch_gate);
  hipLaunchKernelGGL(k_sum_d, dim3(1), dim3(64), 0, st, (const double*)dscratch, nb, dscratch + nb, g_launch_gate);
  hipLaunchKernelGGL(k_mlp_bwd_act, dim3((B + FR * FWV - 1) / (FR * FWV)), dim3(64 * FWV), 0, st, Pb,
                     (const float*)H1, (const float*)H2, (const float*)H3, (const float*)dO, B,
                     D1, D2, D3, g_launch_gate);
  const int nchunk = (B + GCH - 1) / GCH;
  hipLaunchKernelGGL(k_mlp_grad_part, dim3(nchunk), dim3(256), 0, st, S, (const float*)H1,
                     (const float*)H2, (const float*)H3, (const float*)dO, (const float*)D1,
                     (const float*)D2, (const float*)D3, B, gpart, g_launch_gate);
  hipLaunchKernelGGL(k_mlp_grad_sum, dim3((NPAR + 255) / 256), dim3(256), 0, st, (const float*)gpart,
                     nchunk, G, g_launch_gate);
  double loss = 0.0;
  if (want_loss) {
    hipMemcpyAsync(&loss, dscratch + nb, sizeof(double), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
  }
  return loss;
}

void precond_adam(float* P, const float* G, float* M, float* V, int step, float lr,
                  hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, float(step)), c2 = 1.0f - std::pow(b2, float(step));
  hipLaunchKernelGGL(k_adam, dim3((NPAR + 255) / 256), dim3(256), 0, st, P, G, M, V, NPAR, lr, b1,
                     b2, c1, c2, g_launch_gate);
}

void precond_gather(int prec, const void* psi, const void* hpsi, const double* eps,
                    const int* idx, int ns, long V, void* bpsi, void* bh, double* beps,
                    float* onehot, hipStream_t st) {
  dim3 grid(64, unsigned(ns * PC_SHELLS));
  if (prec == 0)
    hipLaunchKernelGGL(k_pc_gather<double2>, grid, dim3(256), 0, st, (const double2*)psi,
                       (const double2*)hpsi, eps, idx, V, (double2*)bpsi, (double2*)bh, beps, onehot, g_launch_gate);
  else
    hipLaunchKernelGGL(k_pc_gather<float2>, grid, dim3(256), 0, st, (const float2*)psi,
                       (const float2*)hpsi, eps, idx, V, (float2*)bpsi, (float2*)bh, beps, onehot, g_launch_gate);
}

void precond_dir(int prec, const void* bpsi, void* bphi, size_t n, hipStream_t st) {
  const unsigned nb = unsigned((n + 255) / 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_pc_dir<double2>, dim3(nb), dim3(256), 0, st, (const double2*)bpsi,
                       (double2*)bphi, n, g_launch_gate);
  else
    hipLaunchKernelGGL(k_pc_dir<float2>, dim3(nb), dim3(256), 0, st, (const float2*)bpsi,
                       (float2*)bphi, n, g_launch_gate);
}

int precond_gram_blocks() { return 128; }

void precond_targets(int prec, const void* bpsi, const void* bh, const void* bd, const void* bhd,
                     const double* beps, int ns, long V, double* part, float* S, hipStream_t st) {
  const int nblk = precond_gram_blocks();
  dim3 grid(nblk, ns);
  if (prec == 0)
    hipLaunchKernelGGL(k_pc_gram<double2>, grid, dim3(256), 0, st, (const double2*)bpsi,
                       (const double2*)bh, (const double2*)bd, (const double2*)bhd, beps, V, part, g_launch_gate);
  else
    hipLaunchKernelGGL(k_pc_gram<float2>, grid, dim3(256), 0, st, (const float2*)bpsi,
                       (const float2*)bh, (const float2*)bd, (const float2*)bhd, beps, V, part, g_launch_gate);
  hipLaunchKernelGGL(k_pc_solve, dim3((ns + 63) / 64), dim3(64), 0, st, (const double*)part, nblk,
                     ns, S, g_launch_gate);
}

size_t precond_gpart_bytes(int rows) {
  return sizeof(float) * size_t(NPAR) * size_t((rows + GCH - 1) / GCH);
}

size_t precond_gram_bytes(int ns) { return sizeof(double) * size_t(ns) * precond_gram_blocks() * NG; }

}  // namespace sky
