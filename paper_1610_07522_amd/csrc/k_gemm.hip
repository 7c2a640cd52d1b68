// Dense complex FP64 products on the FP64 matrix cores (MFMA 16x16x4).
//
// Sec. 3.3.1: the overlap I = <phi|phi> and subspace Hamiltonian
// H = <phi|h phi> are inner products of all state pairs, computed for the
// lower triangle only (Fig. 3).  Sec. 3.3.3: the orthonormalised, diagonal
// states are built with one product psi = phi (C Z) (step 3e).
//
// Tiles, operand staging and the three-product complex scheme are in
// mfma_f64.h.
#include <algorithm>

#include "mfma_f64.h"
#include "sky_kernels.h"

namespace sky {

namespace {
using mfma::Acc;
using mfma::GT;
using mfma::KC;
using mfma::KP;
using mfma::TM;

// Lower-triangle tile pair number p -> (ta, tb), ta >= tb.
__device__ inline void tri_pair(int p, int& ta, int& tb) {
  int a = int((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= p) ++a;
  while (a * (a + 1) / 2 > p) --a;
  ta = a;
  tb = p - a * (a + 1) / 2;
}

// ----------------------------------------------------------- overlap (lower)
// part[(z*npair + pair)*split + s][64*64] = sum over chunk s of conj(A) B^T.
__global__ void __launch_bounds__(GT)
k_overlap_lower(const double2* __restrict__ A, const double2* __restrict__ B0,
                const double2* __restrict__ B1, int m, long k, int split, double2* __restrict__ part, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double2 sA[TM * KP];
  __shared__ double2 sB[TM * KP];
  const int npair = gridDim.x;
  const int pair = blockIdx.x, s = blockIdx.y, z = blockIdx.z;
  const double2* B = z ? B1 : B0;
  int ta, tb;
  tri_pair(pair, ta, tb);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long nck = k / KC;
  const long c0 = nck * s / split, c1 = nck * (s + 1) / split;
  // loader: thread -> (row, 4 consecutive complex); contraction index kk of a
  // row is stored at mfma::kperm(kk), so that the 8 lanes of an LDS store
  // cycle (2 rows x 4 threads) meet 8 different bank groups
  const int lrow = tid >> 2, lk = (tid & 3) * 4;
  const int ga = ta * TM + lrow, gb = tb * TM + lrow;
  // chunk c + 1 is loaded into registers while chunk c is multiplied
  double2 ra[4], rb[4];
  auto load = [&](long c) {
    const long k0 = c * KC + lk;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ra[e] = ga < m ? A[size_t(ga) * k + k0 + e] : make_double2(0, 0);
      rb[e] = gb < m ? B[size_t(gb) * k + k0 + e] : make_double2(0, 0);
    }
  };
  Acc acc;
  mfma::zero(acc);
  if (c0 < c1) load(c0);
  for (long c = c0; c < c1; ++c) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      sA[lrow * KP + mfma::kperm(lk + e)] = ra[e];
      sB[lrow * KP + mfma::kperm(lk + e)] = rb[e];
    }
    __syncthreads();
    if (c + 1 < c1) load(c + 1);
    mfma::tile<true, true>(acc, sA, sB, wm, wn, lane);
    __syncthreads();
  }
  double2* out = part + (size_t(z) * npair + pair) * split * TM * TM + size_t(s) * TM * TM;
  mfma::foreach(acc, wm, wn, lane, [&](int row, int col, double re, double im) {
    out[row * TM + col] = make_double2(re, im);
  });
}

// C[a][b] = scale * sum_s part[..][s][..] for the lower tiles.
__global__ void k_overlap_reduce(const double2* __restrict__ part, int npair, int split, int m,
                                 double scale, double2* __restrict__ C0, double2* __restrict__ C1, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int pair = blockIdx.x, z = blockIdx.y;
  double2* C = z ? C1 : C0;
  int ta, tb;
  tri_pair(pair, ta, tb);
  const double2* p = part + (size_t(z) * npair + pair) * split * TM * TM;
  for (int e = threadIdx.x; e < TM * TM; e += blockDim.x) {
    int row = ta * TM + e / TM, col = tb * TM + e % TM;
    if (row >= m || col >= m) continue;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < split; ++s) {
      double2 v = p[size_t(s) * TM * TM + e];
      re += v.x;
      im += v.y;
    }
    C[size_t(row) * m + col] = make_double2(scale * re, scale * im);
  }
}

__global__ void k_hermitian_fill(double2* __restrict__ C, int m, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int row = blockIdx.y * 16 + threadIdx.y, col = blockIdx.x * 16 + threadIdx.x;
  if (row >= m || col >= m) return;
  if (col > row) {
    double2 v = C[size_t(col) * m + row];
    C[size_t(row) * m + col] = make_double2(v.x, -v.y);
  } else if (col == row) {
    C[size_t(row) * m + col].y = 0.0;
  }
}

// ----------------------------------------------------------- combine
// Y[b][v] = sum_a U[a][b] X[a][v]: M = b (rows of Y), N = v, K = a.
__global__ void __launch_bounds__(GT)
k_combine(const double2* __restrict__ X, const double2* __restrict__ U, double2* __restrict__ Y,
          int m, long k, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double2 sA[TM * KP];   // [b][a]
  __shared__ double2 sB[TM * KP];   // [v][a]
  const long v0 = long(blockIdx.x) * TM;
  const int b0 = blockIdx.y * TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // loader: thread -> (a within chunk = tid/16, columns lc + 16 e): 16 lanes
  // read 256 contiguous bytes, and the transposed LDS stores of 8 lanes land
  // in 8 different bank groups (KP odd)
  const int la = tid >> 4, lc = tid & 15;
  // chunk a0 + KC is loaded into registers while chunk a0 is multiplied
  double2 ru[4], rx[4];
  auto load = [&](int a0) {
    const int a = a0 + la;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int col = lc + 16 * e, b = b0 + col;
      ru[e] = (a < m && b < m) ? U[size_t(a) * m + b] : make_double2(0, 0);
      rx[e] = (a < m) ? X[size_t(a) * k + v0 + col] : make_double2(0, 0);
    }
  };
  Acc acc;
  mfma::zero(acc);
  if (m > 0) load(0);
  for (int a0 = 0; a0 < m; a0 += KC) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int col = lc + 16 * e;
      sA[col * KP + la] = ru[e];
      sB[col * KP + la] = rx[e];
    }
    __syncthreads();
    if (a0 + KC < m) load(a0 + KC);
    mfma::tile<false>(acc, sA, sB, wm, wn, lane);
    __syncthreads();
  }
  mfma::foreach(acc, wm, wn, lane, [&](int row, int col, double re, double im) {
    const int b = b0 + row;
    if (b < m) Y[size_t(b) * k + v0 + col] = make_double2(re, im);
  });
}

// ----------------------------------------------------------- square products
// C = op(A) op(B), op 0 = N, 1 = conjugate transpose; all m x m row-major.
// With lower, a product known to be Hermitian: only tiles on or below the
// diagonal are computed, and the caller mirrors the strictly upper part.
// Grid (column tiles, row tiles, split): workgroup z sums the contraction
// chunks [nk z / split, nk (z+1) / split) and writes C + z m^2 (split > 1:
// partials, reduced in order by k_sum_splits).  Each operand is loaded along
// its contiguous index (op N of B and op H of A read rows of 64 columns), one
// chunk ahead into registers.
template <int OPA, int OPB>
__global__ void __launch_bounds__(GT)
k_gemm_square(const double2* __restrict__ A, const double2* __restrict__ B,
              double2* __restrict__ C, int m, int split, int lower, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double2 sA[TM * KP];   // [row][k] of op(A)
  __shared__ double2 sB[TM * KP];   // [col][k] of op(B)
  constexpr int NE = TM * KC / GT;  // elements per thread and operand
  if (lower && blockIdx.x > blockIdx.y) return;   // Hermitian product: lower tiles only
  const int r0 = blockIdx.y * TM, c0 = blockIdx.x * TM, sp = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int nk = (m + KC - 1) / KC;
  const int kc0 = int((long(nk) * sp) / split), kc1 = int((long(nk) * (sp + 1)) / split);
  // (t, kk) of element q: t = tile row / column, kk = contraction index
  auto idxA = [&](int q, int& t, int& kk) {
    const int e = tid + q * GT;
    if (OPA == 0) { t = e / KC; kk = e % KC; } else { t = e % TM; kk = e / TM; }
  };
  auto idxB = [&](int q, int& t, int& kk) {
    const int e = tid + q * GT;
    if (OPB == 0) { t = e % TM; kk = e / TM; } else { t = e / KC; kk = e % KC; }
  };
  double2 ra[NE], rb[NE];
  auto load = [&](int kc) {
    const int k0 = kc * KC;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      int t, kk;
      idxA(q, t, kk);
      const int r = r0 + t, kg = k0 + kk;
      double2 v = make_double2(0, 0);
      if (r < m && kg < m) {
        if (OPA == 0) v = A[size_t(r) * m + kg];
        else { v = A[size_t(kg) * m + r]; v.y = -v.y; }
      }
      ra[q] = v;
      idxB(q, t, kk);
      const int c = c0 + t, kb = k0 + kk;
      v = make_double2(0, 0);
      if (c < m && kb < m) {
        if (OPB == 0) v = B[size_t(kb) * m + c];
        else { v = B[size_t(c) * m + kb]; v.y = -v.y; }
      }
      rb[q] = v;
    }
  };
  Acc acc;
  mfma::zero(acc);
  if (kc0 < kc1) load(kc0);
  for (int kc = kc0; kc < kc1; ++kc) {
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      int t, kk;
      idxA(q, t, kk);
      sA[t * KP + kk] = ra[q];
      idxB(q, t, kk);
      sB[t * KP + kk] = rb[q];
    }
    __syncthreads();
    if (kc + 1 < kc1) load(kc + 1);
    mfma::tile<false>(acc, sA, sB, wm, wn, lane);
    __syncthreads();
  }
  double2* out = C + size_t(sp) * m * m;
  mfma::foreach(acc, wm, wn, lane, [&](int row, int col, double re, double im) {
    const int r = r0 + row, c = c0 + col;
    if (r < m && c < m) out[size_t(r) * m + c] = make_double2(re, im);
  });
}

// C[e] = sum_s part[s][e], in order.
__global__ void k_sum_splits(const double2* __restrict__ part, int split, size_t n,
                             double2* __restrict__ C, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double2 acc = part[e];
  for (int s = 1; s < split; ++s) {
    const double2 v = part[size_t(s) * n + e];
    acc.x += v.x;
    acc.y += v.y;
  }
  C[e] = acc;
}

// Contraction splits of the square products: enough workgroups for ~4 per
// CU (tile counts such as 625 = 25^2 otherwise leave a long last round);
// herm: only the nt (nt + 1) / 2 lower tiles are live.
int square_split(int m, int herm) {
  if (m <= 0) return 1;   // empty species: nothing to split
  const int nt = (m + TM - 1) / TM;
  const int nk = (m + KC - 1) / KC;
  const int tiles = herm ? nt * (nt + 1) / 2 : nt * nt;
  int split = (1024 + tiles - 1) / tiles;
  if (split > 8) split = 8;
  if (split > nk / 2) split = nk / 2;
  if (split < 1) split = 1;
  return split;
}

int overlap_split(int m, long k) {
  if (m <= 0) return 1;
  const int nt = (m + TM - 1) / TM;
  const int npair = nt * (nt + 1) / 2;
  long nck = k / KC;
  int split = (2048 + 2 * npair - 1) / (2 * npair);
  if (split < 1) split = 1;
  if (split > nck) split = int(nck);
  if (split > 64) split = 64;
  return split;
}
}  // namespace

// Split-K factors tried by the autotuner: half, default and double.
int overlap_split_candidates(int m, long k, int* out) {
  const int d = overlap_split(m, k);
  const long nck = k / KC;
  int n = 0;
  for (int c : {d / 2, d, 2 * d})
    if (c >= 1 && c <= 64 && c <= nck && (n == 0 || out[n - 1] != c)) out[n++] = c;
  return n;
}

size_t overlap_scratch_bytes(int m, long k) {
  const int nt = (m + TM - 1) / TM;
  const int npair = nt * (nt + 1) / 2;
  int c[3];
  const int nc = overlap_split_candidates(m, k, c);
  int split = 1;
  for (int i = 0; i < nc; ++i) split = std::max(split, c[i]);
  return size_t(split) * 2 * npair * TM * TM * sizeof(double2);
}

void overlap_lower(const void* A, const void* B0, const void* B1, int m, long k, double scale,
                   void* C0, void* C1, void* part, hipStream_t st, hipEvent_t* ev, int split_req) {
  if (m <= 0) return;
  const int nt = (m + TM - 1) / TM;
  const int npair = nt * (nt + 1) / 2;
  const int split = split_req > 0 ? split_req : overlap_split(m, k);
  const int nz = B1 ? 2 : 1;
  if (ev) hipEventRecord(ev[0], st);
  hipLaunchKernelGGL(k_overlap_lower, dim3(npair, split, nz), dim3(GT), 0, st,
                     (const double2*)A, (const double2*)B0, (const double2*)B1, m, k, split,
                     (double2*)part, g_launch_gate);
  if (ev) hipEventRecord(ev[1], st);
  overlap_reduce(part, npair, split, m, scale, C0, C1, nz, st);
}

void overlap_reduce(const void* part, int npair, int split, int m, double scale, void* C0,
                    void* C1, int nz, hipStream_t st) {
  hipLaunchKernelGGL(k_overlap_reduce, dim3(npair, nz), dim3(256), 0, st, (const double2*)part,
                     npair, split, m, scale, (double2*)C0, (double2*)C1, g_launch_gate);
}

void hermitian_fill(void* C, int m, hipStream_t st) {
  if (m <= 0) return;
  dim3 grid((m + 15) / 16, (m + 15) / 16), block(16, 16);
  hipLaunchKernelGGL(k_hermitian_fill, grid, block, 0, st, (double2*)C, m, g_launch_gate);
}

void combine(const void* X, const void* U, void* Y, int m, long k, hipStream_t st) {
  if (m <= 0) return;
  dim3 grid(unsigned(k / TM), (m + TM - 1) / TM);
  hipLaunchKernelGGL(k_combine, grid, dim3(GT), 0, st, (const double2*)X, (const double2*)U,
                     (double2*)Y, m, k, g_launch_gate);
}

// Split-K factors tried by the autotuner for square products of size m.
int square_split_candidates(int m, int* out) {
  const int nk = (m + KC - 1) / KC;
  int n = 0;
  for (int c : {1, 2, 4, 8})
    if (c == 1 || c <= nk / 2) out[n++] = c;
  return n;
}

size_t gemm_square_scratch_bytes(int m) {
  int c[4];
  const int nc = square_split_candidates(m, c);
  int split = std::max(square_split(m, 0), square_split(m, 1));
  for (int i = 0; i < nc; ++i) split = std::max(split, c[i]);
  return split > 1 ? size_t(split) * m * m * sizeof(double2) : 0;
}

void gemm_square(const void* A, int opA, const void* B, int opB, void* C, int m, hipStream_t st,
                 void* part, int herm, int split_req) {
  if (m <= 0) return;
  const int split = !part ? 1 : (split_req > 0 ? split_req : square_split(m, herm));
  dim3 grid((m + TM - 1) / TM, (m + TM - 1) / TM, split);
  auto a = (const double2*)A;
  auto b = (const double2*)B;
  auto c = (double2*)(split > 1 ? part : C);
  if (opA == 0 && opB == 0) hipLaunchKernelGGL((k_gemm_square<0, 0>), grid, dim3(GT), 0, st, a, b, c, m, split, herm, g_launch_gate);
  else if (opA == 0 && opB == 1) hipLaunchKernelGGL((k_gemm_square<0, 1>), grid, dim3(GT), 0, st, a, b, c, m, split, herm, g_launch_gate);
  else if (opA == 1 && opB == 0) hipLaunchKernelGGL((k_gemm_square<1, 0>), grid, dim3(GT), 0, st, a, b, c, m, split, herm, g_launch_gate);
  else hipLaunchKernelGGL((k_gemm_square<1, 1>), grid, dim3(GT), 0, st, a, b, c, m, split, herm, g_launch_gate);
  if (split > 1) {
    const size_t n = size_t(m) * m;
    hipLaunchKernelGGL(k_sum_splits, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st,
                       (const double2*)part, split, n, (double2*)C, g_launch_gate);
  }
  if (herm) hermitian_fill(C, m, st);
}

}  // namespace sky
