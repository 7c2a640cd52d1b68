// Mixed-precision subspace products: complex64 operands on the BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16) with the three-way BF16 split.
//
// Every FP32 component x is split once, while a tile is staged in LDS, into
// x = x0 + x1 + x2 (BF16 each, round to nearest even; the residuals are
// exact in FP32).  A real product x*y keeps the six terms
// x0y0 + x0y1 + x1y0 + x0y2 + x2y0 + x1y1, which carries FP32 accuracy
// (the dropped terms are O(2^-24) relative).  MFMA accumulation is FP32 over
// runs of FLUSH*KB contraction elements, then folded into FP64 registers;
// split-K partials are reduced in FP64.  Output of the overlap products is
// FP64 (it feeds the FP64 Cholesky / eigensolver); the recombination writes
// complex64 states.
//
// Sec. 3.3.1 (I and H, lower triangles, Fig. 3) and Sec. 3.3.3 (psi = phi U).
#include "sky_kernels.h"

namespace sky {

namespace {
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64;       // output tile
constexpr int KB = 32;       // contraction elements per MFMA step
constexpr int FLUSH = 8;     // steps accumulated in FP32 before folding into FP64
constexpr int NP = 6;        // split planes: (part re/im) x (split 0..2)
constexpr int RS = KB + 8;   // padded LDS row (bf16 elements); 80 bytes
constexpr int GT = 256;

// BF16 round-to-nearest-even of x, returned as the bit pattern.
__device__ inline unsigned short bf16_bits(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_value(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

// x -> three BF16 parts (bit patterns).
__device__ inline void split3(float x, unsigned short& s0, unsigned short& s1, unsigned short& s2) {
  s0 = bf16_bits(x);
  float r1 = x - bf16_value(s0);
  s1 = bf16_bits(r1);
  float r2 = r1 - bf16_value(s1);
  s2 = bf16_bits(r2);
}

// Plane index: part (0 re, 1 im) * 3 + split.
__device__ inline int plane(int part, int s) { return part * 3 + s; }

// LDS tile: [plane][row][RS] bf16 bit patterns.
struct Tile {
  unsigned short v[NP][TM][RS];
};

// Store the splits of complex value z at (row, k) of a tile.
__device__ inline void put(Tile& t, int row, int k, float2 z) {
  unsigned short a0, a1, a2, b0, b1, b2;
  split3(z.x, a0, a1, a2);
  split3(z.y, b0, b1, b2);
  t.v[0][row][k] = a0; t.v[1][row][k] = a1; t.v[2][row][k] = a2;
  t.v[3][row][k] = b0; t.v[4][row][k] = b1; t.v[5][row][k] = b2;
}

__device__ inline bf8 ld8(const Tile& t, int p, int row, int k8) {
  u4 u = *reinterpret_cast<const u4*>(&t.v[p][row][k8]);
  return __builtin_bit_cast(bf8, u);
}
__device__ inline bf8 neg8(bf8 x) {
  u4 u = __builtin_bit_cast(u4, x);
  u ^= u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  return __builtin_bit_cast(bf8, u);
}

struct Acc32 {
  f4 re[2][2], im[2][2];
};
struct Acc64 {
  double re[2][2][4], im[2][2][4];
};

__device__ inline void zero32(Acc32& a) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) { a.re[i][j] = f4{0, 0, 0, 0}; a.im[i][j] = f4{0, 0, 0, 0}; }
}
__device__ inline void zero64(Acc64& a) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) { a.re[i][j][e] = 0.0; a.im[i][j][e] = 0.0; }
}
__device__ inline void fold(Acc64& d, Acc32& s) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        d.re[i][j][e] += double(s.re[i][j][e]);
        d.im[i][j][e] += double(s.im[i][j][e]);
      }
      s.re[i][j] = f4{0, 0, 0, 0};
      s.im[i][j] = f4{0, 0, 0, 0};
    }
}

#define MF(a, b, c) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0)

// acc += op(A) B^T over one KB step; A rows = tile rows of sA, B cols = rows
// of sB; op(A) = conj(A) if CONJA.  Six split products per real product.
template <bool CONJA>
__device__ inline void step(Acc32& acc, const Tile& sA, const Tile& sB, int wm, int wn, int lane) {
  const int r = lane & 15, k8 = (lane >> 4) * 8;
  bf8 ar[2][3], ai[2][3], br[2][3], bi[2][3];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      ar[i][s] = ld8(sA, plane(0, s), wm * 32 + i * 16 + r, k8);
      ai[i][s] = ld8(sA, plane(1, s), wm * 32 + i * 16 + r, k8);
      if (CONJA) ai[i][s] = neg8(ai[i][s]);
    }
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      br[j][s] = ld8(sB, plane(0, s), wn * 32 + j * 16 + r, k8);
      bi[j][s] = ld8(sB, plane(1, s), wn * 32 + j * 16 + r, k8);
    }
  // split pairs (p, q): 00 01 10 02 20 11
  constexpr int P[6] = {0, 0, 1, 0, 2, 1};
  constexpr int Q[6] = {0, 1, 0, 2, 0, 1};
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const int p = P[t], q = Q[t];
        // re += ar br - ai bi ; im += ar bi + ai br   (ai already negated for conj)
        MF(ar[i][p], br[j][q], acc.re[i][j]);
        MF(neg8(ai[i][p]), bi[j][q], acc.re[i][j]);
        MF(ar[i][p], bi[j][q], acc.im[i][j]);
        MF(ai[i][p], br[j][q], acc.im[i][j]);
      }
}
#undef MF

// Output element of register e of lane l in a 16x16 block (measured):
// row 4*(l/16) + e, column l%16.
template <typename F>
__device__ inline void foreach64(const Acc64& acc, int wm, int wn, int lane, F f) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wm * 32 + i * 16 + 4 * (lane >> 4) + e;
        const int col = wn * 32 + j * 16 + (lane & 15);
        f(row, col, acc.re[i][j][e], acc.im[i][j][e]);
      }
}

__device__ inline void tri_pair(int p, int& ta, int& tb) {
  int a = int((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= p) ++a;
  while (a * (a + 1) / 2 > p) --a;
  ta = a;
  tb = p - a * (a + 1) / 2;
}

// part[(z*npair + pair)*split + s][64*64] (FP64) = sum over chunk s of conj(A) B^T.
__global__ void __launch_bounds__(GT)
k_overlap_lower_mixed(const float2* __restrict__ A, const float2* __restrict__ B0,
                      const float2* __restrict__ B1, int m, long k, int split,
                      double2* __restrict__ part) {
  __shared__ Tile sA, sB;
  const int npair = gridDim.x;
  const int pair = blockIdx.x, s = blockIdx.y, z = blockIdx.z;
  const float2* B = z ? B1 : B0;
  int ta, tb;
  tri_pair(pair, ta, tb);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long nst = k / KB;
  const long c0 = nst * s / split, c1 = nst * (s + 1) / split;
  // loader: thread -> (row = tid/4, 8 consecutive complex at (tid%4)*8)
  const int lrow = tid >> 2, lk = (tid & 3) * 8;
  const int ga = ta * TM + lrow, gb = tb * TM + lrow;
  Acc32 acc;
  Acc64 tot;
  zero32(acc);
  zero64(tot);
  int nacc = 0;
  for (long c = c0; c < c1; ++c) {
    const long k0 = c * KB + lk;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      put(sA, lrow, lk + e, ga < m ? A[size_t(ga) * k + k0 + e] : make_float2(0, 0));
      put(sB, lrow, lk + e, gb < m ? B[size_t(gb) * k + k0 + e] : make_float2(0, 0));
    }
    __syncthreads();
    step<true>(acc, sA, sB, wm, wn, lane);
    __syncthreads();
    if (++nacc == FLUSH) { fold(tot, acc); nacc = 0; }
  }
  fold(tot, acc);
  double2* out = part + (size_t(z) * npair + pair) * split * TM * TM + size_t(s) * TM * TM;
  foreach64(tot, wm, wn, lane, [&](int row, int col, double re, double im) {
    out[row * TM + col] = make_double2(re, im);
  });
}

// Y[b][v] = sum_a U[a][b] X[a][v], X and Y complex64, U FP64 (m x m).
__global__ void __launch_bounds__(GT)
k_combine_mixed(const float2* __restrict__ X, const double2* __restrict__ U,
                float2* __restrict__ Y, int m, long k) {
  __shared__ Tile sA, sB;   // sA: [b][a], sB: [v][a]
  const long v0 = long(blockIdx.x) * TM;
  const int b0 = blockIdx.y * TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // loader: thread -> (a within step = tid/8, 8 consecutive columns)
  const int la = tid >> 3, lc = (tid & 7) * 8;
  Acc32 acc;
  Acc64 tot;
  zero32(acc);
  zero64(tot);
  int nacc = 0;
  for (int a0 = 0; a0 < m; a0 += KB) {
    const int a = a0 + la;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int b = b0 + lc + e;
      float2 u = make_float2(0, 0);
      if (a < m && b < m) {
        double2 ud = U[size_t(a) * m + b];
        u = make_float2(float(ud.x), float(ud.y));
      }
      put(sA, lc + e, la, u);
      put(sB, lc + e, la, a < m ? X[size_t(a) * k + v0 + lc + e] : make_float2(0, 0));
    }
    __syncthreads();
    step<false>(acc, sA, sB, wm, wn, lane);
    __syncthreads();
    if (++nacc == FLUSH) { fold(tot, acc); nacc = 0; }
  }
  fold(tot, acc);
  foreach64(tot, wm, wn, lane, [&](int row, int col, double re, double im) {
    const int b = b0 + row;
    if (b < m) Y[size_t(b) * k + v0 + col] = make_float2(float(re), float(im));
  });
}

int overlap_split_mixed(int m, long k) {
  const int nt = (m + TM - 1) / TM;
  const int npair = nt * (nt + 1) / 2;
  long nst = k / KB;
  int split = (2048 + 2 * npair - 1) / (2 * npair);
  if (split < 1) split = 1;
  if (split > nst) split = int(nst);
  if (split > 64) split = 64;
  return split;
}
}  // namespace

size_t overlap_scratch_bytes_mixed(int m, long k) {
  const int nt = (m + TM - 1) / TM;
  const int npair = nt * (nt + 1) / 2;
  return size_t(overlap_split_mixed(m, k)) * 2 * npair * TM * TM * sizeof(double2);
}

void overlap_lower_mixed(const void* A, const void* B0, const void* B1, int m, long k,
                         double scale, void* C0, void* C1, void* part, hipStream_t st,
                         hipEvent_t* ev) {
  if (m <= 0) return;
  const int nt = (m + TM - 1) / TM;
  const int npair = nt * (nt + 1) / 2;
  const int split = overlap_split_mixed(m, k);
  const int nz = B1 ? 2 : 1;
  if (ev) hipEventRecord(ev[0], st);
  hipLaunchKernelGGL(k_overlap_lower_mixed, dim3(npair, split, nz), dim3(GT), 0, st,
                     (const float2*)A, (const float2*)B0, (const float2*)B1, m, k, split,
                     (double2*)part);
  if (ev) hipEventRecord(ev[1], st);
  overlap_reduce(part, npair, split, m, scale, C0, C1, nz, st);
}

void combine_mixed(const void* X, const void* U, void* Y, int m, long k, hipStream_t st) {
  if (m <= 0) return;
  dim3 grid(unsigned(k / TM), (m + TM - 1) / TM);
  hipLaunchKernelGGL(k_combine_mixed, grid, dim3(GT), 0, st, (const float2*)X,
                     (const double2*)U, (float2*)Y, m, k);
}

}  // namespace sky
