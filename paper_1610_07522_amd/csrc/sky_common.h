// Common device/host definitions of the Sky3D damped-gradient library.
//
// Spinor layout everywhere: [state][spin][z][y][x], complex interleaved
// (re, im), x fastest.  Real fields: [z][y][x].
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace sky {

// ------------------------------------------------------------------ complex
template <typename T> struct cpx {
  T re, im;
};

template <typename T> __host__ __device__ inline cpx<T> mk(T r, T i) { return {r, i}; }
template <typename T> __host__ __device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ inline cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
// multiply by i
template <typename T> __host__ __device__ inline cpx<T> mul_i(cpx<T> a) { return {-a.im, a.re}; }
template <typename T> __host__ __device__ inline T norm2(cpx<T> a) { return a.re * a.re + a.im * a.im; }

// ------------------------------------------------------------------ grids
// Supported cubic grid sizes and their two-stage factorisation N = R1 * R2.
template <int N> struct Fact;
template <> struct Fact<8>  { static constexpr int R1 = 2, R2 = 4; };
template <> struct Fact<16> { static constexpr int R1 = 4, R2 = 4; };
template <> struct Fact<24> { static constexpr int R1 = 4, R2 = 6; };
template <> struct Fact<32> { static constexpr int R1 = 4, R2 = 8; };
template <> struct Fact<48> { static constexpr int R1 = 6, R2 = 8; };
template <> struct Fact<64> { static constexpr int R1 = 8, R2 = 8; };

// Box geometry and spectral constants handed to every kernel by value.
struct GridArgs {
  double dx;      // spacing (fm), equal on all axes
  double dV;      // dx^3
  double kunit;   // 2 pi / L
  // Bloch shift theta_m / L (fm^-1) of the states' wave numbers along x, y, z
  // (twisted boundary conditions; 0 = periodic).  Derivatives of states use
  // i (k_m + tw[m]); real fields are periodic and ignore it.
  double tw[3];
};

// |k| shells of the learned preconditioner: S equal-width shells of |k| up
// to the corner |k|max = sqrt(3) (N/2) kunit of the Brillouin zone.  With
// k = kunit (a, b, c) and m2 = a^2 + b^2 + c^2, shell s >= j exactly when
// |k| / |k|max >= j / S, i.e. 4 S^2 m2 >= 3 j^2 N^2: integer arithmetic, so
// the shell of a mode does not depend on rounding.
constexpr int PC_SHELLS = 8;
__host__ __device__ inline int k_shell(int m2, int n) {
  int s = 0;
#pragma unroll
  for (int j = 1; j < PC_SHELLS; ++j)
    s += (3 * j * j * n * n <= 4 * PC_SHELLS * PC_SHELLS * m2) ? 1 : 0;
  return s;
}

// Mean field of one species (device pointers, FP64 fields [z][y][x]).
struct MeanFieldPtrs {
  const double* U;
  const double* B;
  const double* W;   // [3][z][y][x]
  // the same fields rounded to FP32 (read by the complex64 kernels, which
  // round every field value to FP32 anyway: half the bytes per read)
  const float* U32;
  const float* B32;
  const float* W32;
};

}  // namespace sky

#define SKY_DISPATCH_N(n, ...)                                 \
  switch (n) {                                                 \
    case 8:  { constexpr int NN = 8;  __VA_ARGS__; } break;    \
    case 16: { constexpr int NN = 16; __VA_ARGS__; } break;    \
    case 24: { constexpr int NN = 24; __VA_ARGS__; } break;    \
    case 32: { constexpr int NN = 32; __VA_ARGS__; } break;    \
    case 48: { constexpr int NN = 48; __VA_ARGS__; } break;    \
    case 64: { constexpr int NN = 64; __VA_ARGS__; } break;    \
    default: break;                                            \
  }
