// 64x64 complex FP64 output tiles on the FP64 matrix cores of gfx950
// (v_mfma_f64_16x16x4f64), shared by the GEMM and linear-algebra kernels.
//
// A workgroup of 4 waves (2x2) owns a 64x64 complex tile; each wave a 32x32
// sub-tile = 2x2 MFMA blocks of 16x16.  Operands are staged in LDS as
// sA[row][k] (M x K) and sB[col][k] (N x K), KC complex values of the
// contraction per stage, rows padded to KP.
//
// Complex products use four real products per term with separate real and
// imaginary accumulators.  (A three-product Gauss form was measured slower:
// these kernels are limited by operand staging, not by MFMA issue, and the
// third accumulator costs occupancy.)
#pragma once

#include <hip/hip_runtime.h>

namespace sky {
namespace mfma {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int TM = 64;      // tile rows / cols
constexpr int KC = 16;      // contraction chunk (complex)
constexpr int KP = KC + 1;  // padded LDS row
constexpr int GT = 256;     // threads

struct Acc {
  d4 re[2][2], im[2][2];
};

__device__ inline void zero(Acc& a) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      a.re[i][j] = d4{0, 0, 0, 0};
      a.im[i][j] = d4{0, 0, 0, 0};
    }
}

// Position in an LDS row of contraction index kk < 16 for loaders that store
// 4 consecutive indices per thread: kk = 4 q + e goes to 2 q + (e >> 1) +
// 8 (e & 1), so that one store (fixed e) of two rows x four threads covers
// the eight 16-byte bank groups of 32 banks (odd KP shifts the second row).
__device__ inline int kperm(int kk) { return (kk >> 1) | ((kk & 1) << 3); }

// acc += op(A) B^T over one KC chunk staged in LDS; A conjugated if CONJA;
// PERM: the rows were stored at kperm positions.
template <bool CONJA, bool PERM = false>
__device__ inline void tile(Acc& acc, const double2* sA, const double2* sB, int wm, int wn,
                            int lane) {
  const int r = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < KC; kk += 4) {
    const int kc = PERM ? kperm(kk + kq) : kk + kq;
    double2 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = sA[(wm * 32 + i * 16 + r) * KP + kc];
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = sB[(wn * 32 + j * 16 + r) * KP + kc];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double ai = CONJA ? -a[i].y : a[i].y;
        // (ar + i ai)(br + i bi) = ar br - ai bi + i (ar bi + ai br)
        acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc.re[i][j], 0, 0, 0);
        acc.re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, b[j].y, acc.re[i][j], 0, 0, 0);
        acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].y, acc.im[i][j], 0, 0, 0);
        acc.im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, b[j].x, acc.im[i][j], 0, 0, 0);
      }
  }
}

// Visit every element of the tile held by this lane: f(row, col, re, im).
// The gfx950 FP64 16x16x4 MFMA returns output row 4*e + lane/16 and column
// lane%16 in register e of each lane (measured with a lane probe).
template <typename F>
__device__ inline void foreach(const Acc& acc, int wm, int wn, int lane, F f) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wm * 32 + i * 16 + 4 * e + (lane >> 4);
        const int col = wn * 32 + j * 16 + (lane & 15);
        f(row, col, acc.re[i][j][e], acc.im[i][j][e]);
      }
}

}  // namespace mfma
}  // namespace sky
