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
constexpr int SB = 16;   // samples per workgroup in the MLP kernels
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

// Forward pass of SB samples per workgroup (128 threads = neurons).  H1..H3
// (may be null) keep the activations for the backward pass; O the outputs.
__global__ void __launch_bounds__(PH)
k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ X, int ldx, int B,
          float* __restrict__ H1, float* __restrict__ H2, float* __restrict__ H3,
          float* __restrict__ O, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ float xs[SB][PIN];
  __shared__ float ha[SB][PH], hb[SB][PH];
  __shared__ float red[SB][PH / 64];
  const int j = threadIdx.x, b0 = blockIdx.x * SB;
  if (j < SB * PIN) {
    const int s = j / PIN, i = j % PIN;
    xs[s][i] = (b0 + s < B) ? X[size_t(b0 + s) * ldx + i] : 0.0f;
  }
  __syncthreads();
  for (int s = 0; s < SB; ++s) {
    float a = P[OB1 + j];
    for (int i = 0; i < PIN; ++i) a += P[OW1 + j * PIN + i] * xs[s][i];
    ha[s][j] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  for (int s = 0; s < SB; ++s) {
    float a = P[OB2 + j];
    for (int i = 0; i < PH; ++i) a += P[OW2 + j * PH + i] * ha[s][i];
    hb[s][j] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  if (H1)
    for (int s = 0; s < SB; ++s)
      if (b0 + s < B) H1[size_t(b0 + s) * PH + j] = ha[s][j];
  __syncthreads();
  for (int s = 0; s < SB; ++s) {
    float a = P[OB3 + j];
    for (int i = 0; i < PH; ++i) a += P[OW3 + j * PH + i] * hb[s][i];
    ha[s][j] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  if (H2)
    for (int s = 0; s < SB; ++s)
      if (b0 + s < B) H2[size_t(b0 + s) * PH + j] = hb[s][j];
  if (H3)
    for (int s = 0; s < SB; ++s)
      if (b0 + s < B) H3[size_t(b0 + s) * PH + j] = ha[s][j];
  for (int s = 0; s < SB; ++s) {
    float v = P[OW4 + j] * ha[s][j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((j & 63) == 0) red[s][j >> 6] = v;
  }
  __syncthreads();
  if (j < SB && b0 + j < B) O[b0 + j] = red[j][0] + red[j][1] + P[OB4];
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

// Backward through the hidden layers for SB samples per workgroup:
// D3 = dL/d(pre3), D2 = dL/d(pre2), D1 = dL/d(pre1) (ReLU masks applied).
__global__ void __launch_bounds__(PH)
k_mlp_bwd_act(const float* __restrict__ P, const float* __restrict__ H1,
              const float* __restrict__ H2, const float* __restrict__ H3,
              const float* __restrict__ dO, int B, float* __restrict__ D1,
              float* __restrict__ D2, float* __restrict__ D3, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ float da[SB][PH], db[SB][PH];
  const int j = threadIdx.x, b0 = blockIdx.x * SB;
  for (int s = 0; s < SB; ++s) {
    const int b = b0 + s;
    float v = 0.0f;
    if (b < B) v = (H3[size_t(b) * PH + j] > 0.0f) ? dO[b] * P[OW4 + j] : 0.0f;
    da[s][j] = v;
    if (b < B) D3[size_t(b) * PH + j] = v;
  }
  __syncthreads();
  for (int s = 0; s < SB; ++s) {
    const int b = b0 + s;
    float v = 0.0f;
    for (int i = 0; i < PH; ++i) v += P[OW3 + i * PH + j] * da[s][i];
    if (b < B) v = (H2[size_t(b) * PH + j] > 0.0f) ? v : 0.0f;
    db[s][j] = v;
    if (b < B) D2[size_t(b) * PH + j] = v;
  }
  __syncthreads();
  for (int s = 0; s < SB; ++s) {
    const int b = b0 + s;
    float v = 0.0f;
    for (int i = 0; i < PH; ++i) v += P[OW2 + i * PH + j] * db[s][i];
    if (b < B) {
      v = (H1[size_t(b) * PH + j] > 0.0f) ? v : 0.0f;
      D1[size_t(b) * PH + j] = v;
    }
  }
}

// Weight gradients: one thread per parameter, sums over the batch in FP32.
__global__ void k_mlp_bwd_w(const float* __restrict__ S, const float* __restrict__ H1,
                            const float* __restrict__ H2, const float* __restrict__ H3,
                            const float* __restrict__ dO, const float* __restrict__ D1,
                            const float* __restrict__ D2, const float* __restrict__ D3, int B,
                            float* __restrict__ G, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPAR) return;
  float acc = 0.0f;
  if (p < OB1) {                 // W1[j][i]: D1[b][j] x[b][i]
    const int j = p / PIN, i = p % PIN;
    for (int b = 0; b < B; ++b) acc += D1[size_t(b) * PH + j] * S[size_t(b) * 6 + i];
  } else if (p < OW2) {          // b1
    const int j = p - OB1;
    for (int b = 0; b < B; ++b) acc += D1[size_t(b) * PH + j];
  } else if (p < OB2) {          // W2[j][i]: D2[b][j] H1[b][i]
    const int q = p - OW2, j = q / PH, i = q % PH;
    for (int b = 0; b < B; ++b) acc += D2[size_t(b) * PH + j] * H1[size_t(b) * PH + i];
  } else if (p < OW3) {
    const int j = p - OB2;
    for (int b = 0; b < B; ++b) acc += D2[size_t(b) * PH + j];
  } else if (p < OB3) {          // W3[j][i]: D3[b][j] H2[b][i]
    const int q = p - OW3, j = q / PH, i = q % PH;
    for (int b = 0; b < B; ++b) acc += D3[size_t(b) * PH + j] * H2[size_t(b) * PH + i];
  } else if (p < OW4) {
    const int j = p - OB3;
    for (int b = 0; b < B; ++b) acc += D3[size_t(b) * PH + j];
  } else if (p < OB4) {          // W4[i]: dO[b] H3[b][i]
    const int i = p - OW4;
    for (int b = 0; b < B; ++b) acc += dO[b] * H3[size_t(b) * PH + i];
  } else {
    for (int b = 0; b < B; ++b) acc += dO[b];
  }
  G[p] = acc;
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
  hipLaunchKernelGGL(k_mlp_fwd, dim3((B + SB - 1) / SB), dim3(PH), 0, st, Pb, X, 6, B, H1, H2,
                     H3, O, g_launch_gate);
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
                         float* D3, float* G, double* dscratch, int want_loss, hipStream_t st) {
  if (B <= 0) return 0.0;
  precond_forward(Pb, S, B, H1, H2, H3, O, st);
  const int nb = (B + 255) / 256;
  hipLaunchKernelGGL(k_mlp_loss, dim3(nb), dim3(256), 0, st, (const float*)O, S, B, wsum, dO,
                     dscratch, g_launch_gate);
  hipLaunchKernelGGL(k_sum_d, dim3(1), dim3(64), 0, st, (const double*)dscratch, nb, dscratch + nb, g_launch_gate);
  hipLaunchKernelGGL(k_mlp_bwd_act, dim3((B + SB - 1) / SB), dim3(PH), 0, st, Pb,
                     (const float*)H1, (const float*)H2, (const float*)H3, (const float*)dO, B,
                     D1, D2, D3, g_launch_gate);
  hipLaunchKernelGGL(k_mlp_bwd_w, dim3((NPAR + 255) / 256), dim3(256), 0, st, S,
                     (const float*)H1, (const float*)H2, (const float*)H3, (const float*)dO,
                     (const float*)D1, (const float*)D2, (const float*)D3, B, G, g_launch_gate);
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

size_t precond_gram_bytes(int ns) { return sizeof(double) * size_t(ns) * precond_gram_blocks() * NG; }

}  // namespace sky
