// Batched radix FFTs along one grid axis, staged through LDS.
//
// Sec. 2.2 of the paper takes every derivative of a wave function with FFTs.
// Here a line of N points (one axis of the box, all spin components) is
// transformed by a two-stage Cooley-Tukey factorisation N = R1 * R2:
//
//   stage A: thread j (< R2) holds the points j + R2*j1 (j1 < R1) in
//            registers, does a length-R1 DFT over j1 and the inter-stage
//            twiddle w_N^(j*k1);
//   exchange through a small per-line LDS buffer;
//   stage B: thread j (< R1) holds the frequencies j + R1*k2 (k2 < R2) and
//            does a length-R2 DFT over k2.
//
// A spectral multiplier is applied to the stage-B registers, and the inverse
// runs the same stages backwards, so a derivative F^-1[m(k) F psi] costs two
// LDS exchanges and returns the result to the same thread/positions that
// loaded the input.  Forward sign: X[k] = sum_n x[n] exp(-2 pi i n k / N);
// the inverse carries the 1/N.
#pragma once

#include "sky_common.h"

namespace sky {

// ---------------------------------------------------------------- small DFTs
// Twiddle exp(-+2 pi i m / R) for R in {6, 8}; forward sign unless INV.
template <typename T, int R, bool INV> __device__ inline cpx<T> tw_small(int m) {
  constexpr T s3 = T(0.86602540378443864676);  // sin(pi/3)
  constexpr T r2 = T(0.70710678118654752440);  // 1/sqrt(2)
  T c = 0, s = 0;  // exp(-2 pi i m / R) = c + i s
  if constexpr (R == 6) {
    const T C[6] = {T(1), T(0.5), T(-0.5), T(-1), T(-0.5), T(0.5)};
    const T S[6] = {T(0), -s3, -s3, T(0), s3, s3};
    c = C[m]; s = S[m];
  } else {
    const T C[8] = {T(1), r2, T(0), -r2, T(-1), -r2, T(0), r2};
    const T S[8] = {T(0), -r2, T(-1), -r2, T(0), r2, T(1), r2};
    c = C[m]; s = S[m];
  }
  return INV ? mk(c, -s) : mk(c, s);
}

template <typename T, int R, bool INV> struct DFT;

template <typename T, bool INV> struct DFT<T, 1, INV> {
  __device__ static inline void run(cpx<T>*) {}
};

template <typename T, bool INV> struct DFT<T, 2, INV> {
  __device__ static inline void run(cpx<T>* v) {
    cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T, bool INV> struct DFT<T, 3, INV> {
  __device__ static inline void run(cpx<T>* v) {
    constexpr T s3 = T(0.86602540378443864676);
    cpx<T> t1 = v[1] + v[2], t2 = v[1] - v[2];
    cpx<T> m = v[0] - T(0.5) * t1;
    cpx<T> it2 = mul_i(t2);                   // i (v1 - v2)
    v[0] = v[0] + t1;
    if (INV) { v[1] = m + s3 * it2; v[2] = m - s3 * it2; }
    else     { v[1] = m - s3 * it2; v[2] = m + s3 * it2; }
  }
};

template <typename T, bool INV> struct DFT<T, 4, INV> {
  __device__ static inline void run(cpx<T>* v) {
    cpx<T> a = v[0] + v[2], b = v[0] - v[2];
    cpx<T> c = v[1] + v[3], d = mul_i(v[1] - v[3]);
    v[0] = a + c;
    v[2] = a - c;
    if (INV) { v[1] = b + d; v[3] = b - d; }
    else     { v[1] = b - d; v[3] = b + d; }
  }
};

// Composite length P*Q: inner DFT_P over x[q + Q p], twiddle, outer DFT_Q.
template <typename T, int P, int Q, bool INV> struct DFTComposite {
  __device__ static inline void run(cpx<T>* v) {
    constexpr int R = P * Q;
    cpx<T> y[Q][P];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
      for (int p = 0; p < P; ++p) y[q][p] = v[q + Q * p];
      DFT<T, P, INV>::run(y[q]);
#pragma unroll
      for (int kp = 1; kp < P; ++kp)
        if (q > 0) y[q][kp] = y[q][kp] * tw_small<T, R, INV>(q * kp);
    }
#pragma unroll
    for (int kp = 0; kp < P; ++kp) {
      cpx<T> z[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) z[q] = y[q][kp];
      DFT<T, Q, INV>::run(z);
#pragma unroll
      for (int kq = 0; kq < Q; ++kq) v[kp + P * kq] = z[kq];
    }
  }
};

template <typename T, bool INV> struct DFT<T, 6, INV> {
  __device__ static inline void run(cpx<T>* v) { DFTComposite<T, 2, 3, INV>::run(v); }
};
template <typename T, bool INV> struct DFT<T, 8, INV> {
  __device__ static inline void run(cpx<T>* v) { DFTComposite<T, 2, 4, INV>::run(v); }
};

// ---------------------------------------------------------------- line engine
// Launch shape of the line kernels for grid size N.
// Lines (pencils) per workgroup: LP = 0 picks the default, otherwise LP.
template <int N, int LP = 0> struct LineCfg {
  static constexpr int R1 = Fact<N>::R1, R2 = Fact<N>::R2;
  static constexpr int RT = R1 > R2 ? R1 : R2;          // threads per line
  static constexpr int LPW = LP ? LP : ((RT == 4) ? 64 : 32);   // lines per workgroup
  static constexpr int THREADS = RT * LPW;
  static_assert((N * N) % LPW == 0, "lines must tile the plane");
  static_assert(THREADS <= 1024, "workgroup too large");
};

// FFT of S spinor components along one line, S in {1, 2}.
// Y is the line's LDS exchange buffer of YSIZE complex values.
template <typename T, int N, int S> struct LineFFT {
  static constexpr int R1 = Fact<N>::R1, R2 = Fact<N>::R2;
  static constexpr int YROW = R2 + 1;                 // padded row
  static constexpr int YSIZE = S * R1 * YROW + 1;     // odd stride between lines

  // va[s][j1] at positions j + R2*j1  ->  vb[s][k2] at frequencies j + R1*k2
  __device__ static inline void forward(cpx<T> (&va)[S][R1], cpx<T> (&vb)[S][R2],
                                        cpx<T>* Y, int j, const cpx<T>* twN) {
    if (j < R2) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        DFT<T, R1, false>::run(va[s]);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
          cpx<T> w = twN[j * k1];
          Y[(s * R1 + k1) * YROW + j] = va[s][k1] * w;
        }
      }
    }
    __syncthreads();
    if (j < R1) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) vb[s][k2] = Y[(s * R1 + j) * YROW + k2];
        DFT<T, R2, false>::run(vb[s]);
      }
    }
    __syncthreads();
  }

  // vb[s][k2] at frequencies j + R1*k2  ->  va[s][j1] at positions j + R2*j1
  __device__ static inline void inverse(cpx<T> (&vb)[S][R2], cpx<T> (&va)[S][R1],
                                        cpx<T>* Y, int j, const cpx<T>* twN) {
    if (j < R1) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        DFT<T, R2, true>::run(vb[s]);
#pragma unroll
        for (int j2 = 0; j2 < R2; ++j2)
          Y[(s * R1 + j) * YROW + j2] = vb[s][j2] * conj(twN[j2 * j]);
      }
    }
    __syncthreads();
    if (j < R2) {
      constexpr T inv_n = T(1) / T(N);
#pragma unroll
      for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) va[s][k1] = Y[(s * R1 + k1) * YROW + j];
        DFT<T, R1, true>::run(va[s]);
#pragma unroll
        for (int j1 = 0; j1 < R1; ++j1) va[s][j1] = inv_n * va[s][j1];
      }
    }
    __syncthreads();
  }

  // In-place spectral derivative i*(k + kshift) along the line, Nyquist kept
  // (k = -N/2); kshift is the Bloch shift of twisted boundary conditions.
  __device__ static inline void deriv(cpx<T> (&va)[S][R1], cpx<T>* Y, int j,
                                      const cpx<T>* twN, T kunit, T kshift = T(0)) {
    cpx<T> vb[S][R2];
    forward(va, vb, Y, j, twN);
    if (j < R1) {
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        int f = j + R1 * k2;
        T k = kunit * T(f < N / 2 ? f : f - N) + kshift;
#pragma unroll
        for (int s = 0; s < S; ++s) vb[s][k2] = mul_i(k * vb[s][k2]);
      }
    }
    inverse(vb, va, Y, j, twN);
  }
};

// Distance in LDS between the exchange buffers of consecutive lines of a
// workgroup (complex values).  Along y and z consecutive lanes hold
// consecutive lines, which the odd YSIZE spreads over the banks.  Along x a
// wave holds 64 / RT lines of RT consecutive threads; for those the strides
// below put the words of every exchange access of a wave in distinct banks,
// for 32 and for 64 banks of 4 bytes and 8- or 16-byte values (counted on
// the CPU for each access of the two stages; N = 24, whose lines straddle
// waves, takes the stride with the fewest shared banks).
template <int N, int S> constexpr int x_line_stride() {
  constexpr int one[6] = {12, 20, 38, 40, 56, 72};     // S = 1
  constexpr int two[6] = {20, 44, 70, 72, 120, 152};   // S = 2
  constexpr int i = N == 8 ? 0 : N == 16 ? 1 : N == 24 ? 2 : N == 32 ? 3 : N == 48 ? 4 : 5;
  return S == 1 ? one[i] : two[i];
}
template <typename T, int N, int S, int DIR> constexpr int line_stride() {
  constexpr int v = DIR == 0 ? x_line_stride<N, S>() : LineFFT<T, N, S>::YSIZE;
  static_assert(v >= S * Fact<N>::R1 * (Fact<N>::R2 + 1), "exchange buffer too small");
  return v;
}

// The same two-stage FFT with the exchange done in place, in the line's own
// N slots: element idx of spin component s lives at base[s * sp + idx * es]
// (es = 1 for a row, the row pitch for a column of an LDS slice).  Stage A
// of thread j writes exactly the slots it loaded (k1 * R2 + j), so only the
// stage boundaries need barriers; the inverse starts with one, since its
// stage-B writes land on slots other threads have just loaded from.  Every
// thread of the workgroup must call these (barriers).
template <typename T, int N, int S> struct LineFFTInPlace {
  static constexpr int R1 = Fact<N>::R1, R2 = Fact<N>::R2;

  // va[s][j1] at positions j + R2*j1  ->  vb[s][k2] at frequencies j + R1*k2
  __device__ static inline void forward(cpx<T> (&va)[S][R1], cpx<T> (&vb)[S][R2], cpx<T>* base,
                                        int sp, int es, int j, const cpx<T>* twN) {
    if (j < R2) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        DFT<T, R1, false>::run(va[s]);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) base[s * sp + (k1 * R2 + j) * es] = va[s][k1] * twN[j * k1];
      }
    }
    __syncthreads();
    if (j < R1) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) vb[s][k2] = base[s * sp + (j * R2 + k2) * es];
        DFT<T, R2, false>::run(vb[s]);
      }
    }
    __syncthreads();
  }

  // vb[s][k2] at frequencies j + R1*k2  ->  va[s][j1] at positions j + R2*j1
  __device__ static inline void inverse(cpx<T> (&vb)[S][R2], cpx<T> (&va)[S][R1], cpx<T>* base,
                                        int sp, int es, int j, const cpx<T>* twN) {
    __syncthreads();
    if (j < R1) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        DFT<T, R2, true>::run(vb[s]);
#pragma unroll
        for (int j2 = 0; j2 < R2; ++j2)
          base[s * sp + (j * R2 + j2) * es] = vb[s][j2] * conj(twN[j2 * j]);
      }
    }
    __syncthreads();
    if (j < R2) {
      constexpr T inv_n = T(1) / T(N);
#pragma unroll
      for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) va[s][k1] = base[s * sp + (k1 * R2 + j) * es];
        DFT<T, R1, true>::run(va[s]);
#pragma unroll
        for (int j1 = 0; j1 < R1; ++j1) va[s][j1] = inv_n * va[s][j1];
      }
    }
    __syncthreads();
  }
};

// exp(-2 pi i m / N), m < N, into LDS (all threads of the block help).
template <typename T, int N> __device__ inline void load_twiddles(cpx<T>* tw) {
  for (int m = threadIdx.x; m < N; m += blockDim.x) {
    double s, c;
    sincospi(-2.0 * double(m) / double(N), &s, &c);
    tw[m] = mk(T(c), T(s));
  }
  __syncthreads();
}

// Geometry of line number L along axis DIR (0 = x, 1 = y, 2 = z):
// offset of its first point and the stride between its points.
template <int N, int DIR> __device__ inline void line_geom(int L, int& base, int& stride,
                                                           int& a, int& b) {
  a = L % N;
  b = L / N;
  if (DIR == 0) { base = b * N * N + a * N; stride = 1; }          // (y, z)
  else if (DIR == 1) { base = b * N * N + a; stride = N; }         // (x, z)
  else { base = b * N + a; stride = N * N; }                       // (x, y)
}

// Thread -> (line within workgroup, role j).  Along x the role varies
// fastest so consecutive threads touch consecutive points; along y and z
// the line varies fastest so consecutive threads touch consecutive x.
template <int N, int DIR, int LP = 0> __device__ inline void thread_role(int t, int& line, int& j) {
  constexpr int RT = LineCfg<N, LP>::RT, LPW = LineCfg<N, LP>::LPW;
  if (DIR == 0) { j = t % RT; line = t / RT; }
  else { j = t / LPW; line = t % LPW; }
}

}  // namespace sky
