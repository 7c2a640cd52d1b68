// Grid kernels on the spinor wave functions: h*psi, the damped gradient
// step, and the local densities.  All are passes over lines of one axis
// (fft_line.h); one workgroup takes LPW lines of one state (h, damping) or of
// a chunk of states (densities).
#include <algorithm>

#include "fft_line.h"
#include "sky_kernels.h"

namespace sky {

// Spin-orbit matrix A_dir = (W x sigma)_dir = ax*sx + ay*sy + az*sz.
// Field value at point r in the kernel's precision: complex64 kernels read
// the FP32 copies (the same rounding as converting the FP64 value).
template <typename T> __device__ inline T fld_U(const MeanFieldPtrs& m, size_t r) {
  if constexpr (sizeof(T) == 4) return m.U32[r]; else return m.U[r];
}
template <typename T> __device__ inline T fld_B(const MeanFieldPtrs& m, size_t r) {
  if constexpr (sizeof(T) == 4) return m.B32[r]; else return m.B[r];
}
template <typename T> __device__ inline T fld_W(const MeanFieldPtrs& m, size_t r) {
  if constexpr (sizeof(T) == 4) return m.W32[r]; else return m.W[r];
}

template <int DIR, typename V> __device__ inline void so_coeffs(V wx, V wy, V wz, V& ax, V& ay, V& az) {
  if (DIR == 0) { ax = 0.0; ay = -wz; az = wy; }
  else if (DIR == 1) { ax = wz; ay = 0.0; az = -wx; }
  else { ax = -wy; ay = wx; az = 0.0; }
}

// (a.sigma) chi for a real 3-vector a.
template <typename T> __device__ inline void sigma_apply(T ax, T ay, T az, cpx<T> u, cpx<T> d,
                                                         cpx<T>& ou, cpx<T>& od) {
  // [[az, ax - i ay], [ax + i ay, -az]]
  cpx<T> xm = mk(ax, -ay), xp = mk(ax, ay);
  ou = az * u + xm * d;
  od = xp * u - az * d;
}

// Workgroup sum of one double per thread (blockDim <= 256), result in thread 0.
__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s += red[w];
  }
  __syncthreads();
  return s;
}

// Largest |component| (real or imaginary part, as float) of the values this
// workgroup wrote, merged into *amax as float bits (non-negative floats
// order like their bit patterns).  Any blockDim; every thread must call it.
__device__ inline void block_amax(float v, unsigned int* amax) {
  __shared__ unsigned int smax;
  if (threadIdx.x == 0) smax = 0u;
  __syncthreads();
  atomicMax(&smax, __float_as_uint(v));
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(amax, smax);
}

template <typename T> __device__ inline float cabs_max(cpx<T> z) {
  return fmaxf(fabsf(float(z.re)), fabsf(float(z.im)));
}

// ------------------------------------------------------------------ h * psi
// One pass adds the DIR part of h:
//   - D(B D psi) + (i/2) [A D psi + D(A psi)]  =  D g + (i/2) A D psi,
//   g = -B D psi + (i/2) A psi,
// plus U psi on the first pass.  The last pass also forms per-workgroup
// partial sums of <psi|h psi> for the Rayleigh quotients.
template <typename T, int N, int DIR, bool FIRST, bool LAST, int LP>
__global__ void __launch_bounds__((LineCfg<N, LP>::THREADS))
k_h_pass(const cpx<T>* __restrict__ psi, cpx<T>* __restrict__ hpsi, MeanFieldPtrs mf,
         GridArgs g, double* __restrict__ eps_part, unsigned int* __restrict__ amax, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using C = LineCfg<N, LP>;
  using F = LineFFT<T, N, 2>;
  constexpr int YS = line_stride<T, N, 2, DIR>();
  constexpr int R1 = C::R1, R2 = C::R2, N3 = N * N * N;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> Ybuf[C::LPW * YS];
  __shared__ double red[4];
  load_twiddles<T, N>(tw);

  int line, j;
  thread_role<N, DIR, LP>(threadIdx.x, line, j);
  const int L = blockIdx.x * C::LPW + line;
  int base, stride, a, b;
  line_geom<N, DIR>(L, base, stride, a, b);
  const size_t soff = size_t(blockIdx.y) * 2 * N3;
  const cpx<T>* p = psi + soff;
  cpx<T>* hp = hpsi + soff;
  cpx<T>* Y = Ybuf + line * YS;
  const T kunit = T(g.kunit);
  const T kshift = T(g.tw[DIR]);

  cpx<T> v[2][R1], d[2][R1];
  if (j < R2) {
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      int r = base + (j + R2 * j1) * stride;
      v[0][j1] = p[r];
      v[1][j1] = p[N3 + r];
      d[0][j1] = v[0][j1];
      d[1][j1] = v[1][j1];
    }
  }
  F::deriv(d, Y, j, tw, kunit, kshift);

  // g (into d) and the accumulated local terms (into acc)
  cpx<T> acc[2][R1];
  if (j < R2) {
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      int r = base + (j + R2 * j1) * stride;
      const T B = fld_B<T>(mf, r);
      T ax, ay, az;
      so_coeffs<DIR>(fld_W<T>(mf, r), fld_W<T>(mf, N3 + r), fld_W<T>(mf, 2 * N3 + r), ax, ay, az);
      cpx<T> au, ad, bu, bd;
      sigma_apply<T>(T(ax), T(ay), T(az), d[0][j1], d[1][j1], au, ad);     // A D psi
      sigma_apply<T>(T(ax), T(ay), T(az), v[0][j1], v[1][j1], bu, bd);     // A psi
      acc[0][j1] = T(0.5) * mul_i(au);
      acc[1][j1] = T(0.5) * mul_i(ad);
      if (FIRST) {
        const T U = fld_U<T>(mf, r);
        acc[0][j1] = acc[0][j1] + U * v[0][j1];
        acc[1][j1] = acc[1][j1] + U * v[1][j1];
      }
      d[0][j1] = T(0.5) * mul_i(bu) - B * d[0][j1];
      d[1][j1] = T(0.5) * mul_i(bd) - B * d[1][j1];
    }
  }
  F::deriv(d, Y, j, tw, kunit, kshift);

  double dot = 0.0;
  float am = 0.0f;
  if (j < R2) {
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      int r = base + (j + R2 * j1) * stride;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        cpx<T> t = acc[s][j1] + d[s][j1];
        if (!FIRST) t = t + hp[s * N3 + r];
        hp[s * N3 + r] = t;
        if (LAST) dot += double(v[s][j1].re) * double(t.re) + double(v[s][j1].im) * double(t.im);
        if (LAST) am = fmaxf(am, cabs_max(t));
      }
    }
  }
  if (LAST && eps_part != nullptr) {
    double sum = block_sum(dot, red);
    if (threadIdx.x == 0) eps_part[size_t(blockIdx.y) * gridDim.x + blockIdx.x] = sum * g.dV;
  }
  if (LAST && amax != nullptr) block_amax(am, amax);
}

// Sum the per-workgroup partials of each state: out[s] = sum_t part[s][t].
__global__ void k_sum_partials(const double* __restrict__ part, int ntile, int nstate,
                               double* __restrict__ out, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nstate) return;
  double acc = 0.0;
  for (int t = 0; t < ntile; ++t) acc += part[size_t(s) * ntile + t];
  out[s] = acc;
}

// ------------------------------------------------------------------ xy planes
// One workgroup holds a z-slice of one state (both spin components, N x N
// points, rows padded to N + 1) in LDS and runs the x lines (rows) and the y
// lines (columns) of a pass on it, so that x and y cost one read and one
// write of the state instead of two each.  Threads: N lines x RT per line.
// Used where slice and exchange buffers fit 80 KB of LDS (two workgroups per
// CU): every grid in complex64 up to 48^3, complex128 up to 32^3.
template <int N> struct PlaneCfg {
  static constexpr int R1 = Fact<N>::R1, R2 = Fact<N>::R2;
  static constexpr int RT = R1 > R2 ? R1 : R2;
  static constexpr int THREADS = N * RT;
  static constexpr int PITCH = N + 1;
  static constexpr int SPIN = N * PITCH;   // one spin component of the slice
};

template <typename T, int N> constexpr int plane_lds(int xs) {
  const int ys = LineFFT<T, N, 2>::YSIZE;
  return (2 * PlaneCfg<N>::SPIN + N * (xs > ys ? xs : ys) + N) * int(sizeof(cpx<T>));
}
// Stride of the h slice kernel's x-line buffers: the bank-spreading x stride
// where the slice still fits 80 KB, else the y lines' stride.
template <typename T, int N> constexpr int plane_xstride() {
  return plane_lds<T, N>(line_stride<T, N, 2, 0>()) <= 80 * 1024 ? line_stride<T, N, 2, 0>()
                                                                 : LineFFT<T, N, 2>::YSIZE;
}
template <typename T, int N> constexpr bool plane_fits() {
  return PlaneCfg<N>::THREADS <= 1024 && plane_lds<T, N>(plane_xstride<T, N>()) <= 80 * 1024;
}
// The damped step's slice kernels exchange in place in the slice (no line
// buffers): half the LDS of the h slices.
template <typename T, int N> constexpr bool damp_slices_fit() {
  return PlaneCfg<N>::THREADS <= 1024 && (2 * PlaneCfg<N>::SPIN + N) * sizeof(cpx<T>) <= 80 * 1024;
}
// Default use: measured on MI355X, the slices win up to 32^3 (damped step
// 16% faster, h psi even or faster); at 48^3 their 80 KB of LDS leaves two
// workgroups per CU and the line passes are faster.  The tuner decides per box.
template <typename T, int N> constexpr bool plane_default() { return plane_fits<T, N>() && N <= 32; }
template <typename T, int N> constexpr bool damp_slice_default() {
  return damp_slices_fit<T, N>() && N <= 32;
}

// Deterministic workgroup sum of one double per thread (any blockDim), using
// buf[blockDim.x] of LDS; the result is returned to thread 0.
__device__ inline double tree_sum(double v, double* buf) {
  buf[threadIdx.x] = v;
  __syncthreads();
  int n = blockDim.x;
  while (n > 1) {
    const int h = (n + 1) / 2;
    if (threadIdx.x < n - h) buf[threadIdx.x] += buf[threadIdx.x + h];
    __syncthreads();
    n = h;
  }
  return buf[0];
}

// The DIR part of h on one line held by this thread (R1 points at grid
// offsets r[j1]): D g + (i/2) A D psi with g = -B D psi + (i/2) A psi.
template <typename T, int N, int DIR>
__device__ inline void h_dir_line(const cpx<T> (&v)[2][Fact<N>::R1], cpx<T> (&out)[2][Fact<N>::R1],
                                  const int (&r)[Fact<N>::R1], cpx<T>* Y, int j,
                                  const cpx<T>* tw, T kunit, T kshift,
                                  const MeanFieldPtrs& mf) {
  using F = LineFFT<T, N, 2>;
  constexpr int R1 = Fact<N>::R1, R2 = Fact<N>::R2, N3 = N * N * N;
  cpx<T> d[2][R1];
#pragma unroll
  for (int j1 = 0; j1 < R1; ++j1) {
    d[0][j1] = v[0][j1];
    d[1][j1] = v[1][j1];
  }
  F::deriv(d, Y, j, tw, kunit, kshift);
  if (j < R2) {
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      const int q = r[j1];
      const T B = fld_B<T>(mf, q);
      T ax, ay, az;
      so_coeffs<DIR>(fld_W<T>(mf, q), fld_W<T>(mf, N3 + q), fld_W<T>(mf, 2 * N3 + q), ax, ay, az);
      cpx<T> au, ad, bu, bd;
      sigma_apply<T>(T(ax), T(ay), T(az), d[0][j1], d[1][j1], au, ad);     // A D psi
      sigma_apply<T>(T(ax), T(ay), T(az), v[0][j1], v[1][j1], bu, bd);     // A psi
      out[0][j1] = T(0.5) * mul_i(au);
      out[1][j1] = T(0.5) * mul_i(ad);
      d[0][j1] = T(0.5) * mul_i(bu) - B * d[0][j1];
      d[1][j1] = T(0.5) * mul_i(bd) - B * d[1][j1];
    }
  }
  F::deriv(d, Y, j, tw, kunit, kshift);
  if (j < R2) {
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      out[0][j1] = out[0][j1] + d[0][j1];
      out[1][j1] = out[1][j1] + d[1][j1];
    }
  }
}

// x and y parts of h psi on slice z = blockIdx.x of state blockIdx.y, added to
// what hpsi holds (the z part and U psi); partial sums of <psi|h psi>.
template <typename T, int N>
__global__ void __launch_bounds__(PlaneCfg<N>::THREADS)
k_h_plane(const cpx<T>* __restrict__ psi, cpx<T>* __restrict__ hpsi, MeanFieldPtrs mf, GridArgs g,
          double* __restrict__ eps_part, unsigned int* __restrict__ amax, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using C = PlaneCfg<N>;
  using F = LineFFT<T, N, 2>;
  constexpr int R1 = C::R1, R2 = C::R2, RT = C::RT, PITCH = C::PITCH, SP = C::SPIN;
  constexpr int N2 = N * N, N3 = N * N2;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> P[2 * SP];
  constexpr int XS = plane_xstride<T, N>(), YS = F::YSIZE;   // x- and y-line buffers
  __shared__ cpx<T> Ybuf[N * (XS > YS ? XS : YS)];
  load_twiddles<T, N>(tw);
  const int zoff = blockIdx.x * N2;
  const size_t soff = size_t(blockIdx.y) * 2 * N3;
  const cpx<T>* p = psi + soff;
  cpx<T>* hp = hpsi + soff;
  constexpr int NIT = (2 * N2 + C::THREADS - 1) / C::THREADS;   // unrolled: loads go out together
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * C::THREADS;
    if (i < 2 * N2) {
      const int s = i / N2, e = i - s * N2;
      P[s * SP + (e / N) * PITCH + e % N] = p[s * N3 + zoff + e];
    }
  }
  __syncthreads();
  const T kunit = T(g.kunit);
  // x lines: row ly, role jx (role fastest: consecutive threads, consecutive x)
  const int jx = threadIdx.x % RT, ly = threadIdx.x / RT;
  cpx<T> vx[2][R1], ax[2][R1];
  int rx[R1];
#pragma unroll
  for (int j1 = 0; j1 < R1; ++j1) {
    const int x = jx + R2 * j1;
    rx[j1] = zoff + ly * N + x;
    if (jx < R2) {
      vx[0][j1] = P[ly * PITCH + x];
      vx[1][j1] = P[SP + ly * PITCH + x];
    }
  }
  h_dir_line<T, N, 0>(vx, ax, rx, Ybuf + ly * XS, jx, tw, kunit, T(g.tw[0]), mf);
  // y lines: column lx (line fastest: consecutive threads, consecutive x)
  const int lx = threadIdx.x % N, jy = threadIdx.x / N;
  cpx<T> vy[2][R1], ay[2][R1];
  int ry[R1];
#pragma unroll
  for (int j1 = 0; j1 < R1; ++j1) {
    const int y = jy + R2 * j1;
    ry[j1] = zoff + y * N + lx;
    if (jy < R2) {
      vy[0][j1] = P[y * PITCH + lx];
      vy[1][j1] = P[SP + y * PITCH + lx];
    }
  }
  __syncthreads();
  if (jx < R2) {
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      P[ly * PITCH + jx + R2 * j1] = ax[0][j1];
      P[SP + ly * PITCH + jx + R2 * j1] = ax[1][j1];
    }
  }
  __syncthreads();
  h_dir_line<T, N, 1>(vy, ay, ry, Ybuf + lx * YS, jy, tw, kunit, T(g.tw[1]), mf);
  double dot = 0.0;
  float am = 0.0f;
  if (jy < R2) {
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      const int y = jy + R2 * j1;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const cpx<T> t = ay[s][j1] + P[s * SP + y * PITCH + lx] + hp[s * N3 + ry[j1]];
        hp[s * N3 + ry[j1]] = t;
        dot += double(vy[s][j1].re) * double(t.re) + double(vy[s][j1].im) * double(t.im);
        am = fmaxf(am, cabs_max(t));
      }
    }
  }
  if (eps_part != nullptr) {
    __syncthreads();   // P is free again: reuse it for the reduction
    const double sum = tree_sum(dot, reinterpret_cast<double*>(P));
    if (threadIdx.x == 0) eps_part[size_t(blockIdx.y) * gridDim.x + blockIdx.x] = sum * g.dV;
  }
  if (amax != nullptr) block_amax(am, amax);
}

// Damped step, first half: r = h psi - eps psi on slice z of state
// blockIdx.y, forward FFTs along x and y, spectrum to out; ||r||^2 partials.
template <typename T, int N>
__global__ void __launch_bounds__(PlaneCfg<N>::THREADS)
k_damp_fwd_xy(const cpx<T>* __restrict__ psi, const cpx<T>* __restrict__ hpsi,
              const double* __restrict__ eps, cpx<T>* __restrict__ out, GridArgs g,
              double* __restrict__ r2_part, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using C = PlaneCfg<N>;
  using F = LineFFTInPlace<T, N, 2>;
  constexpr int R1 = C::R1, R2 = C::R2, RT = C::RT, PITCH = C::PITCH, SP = C::SPIN;
  constexpr int N2 = N * N, N3 = N * N2;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> P[2 * SP];
  load_twiddles<T, N>(tw);
  const int zoff = blockIdx.x * N2;
  const size_t soff = size_t(blockIdx.y) * 2 * N3;
  const T e = T(eps[blockIdx.y]);
  double r2 = 0.0;
  constexpr int NIT = (2 * N2 + C::THREADS - 1) / C::THREADS;   // unrolled: loads go out together
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * C::THREADS;
    if (i < 2 * N2) {
      const int s = i / N2, q = i - s * N2;
      const size_t o = soff + s * N3 + zoff + q;
      const cpx<T> res = hpsi[o] - e * psi[o];
      r2 += double(res.re) * double(res.re) + double(res.im) * double(res.im);
      P[s * SP + (q / N) * PITCH + q % N] = res;
    }
  }
  __syncthreads();
  {  // x lines, in place (row ly; rows fastest across the lanes, whose odd
     // pitch puts a wave's accesses in distinct LDS banks)
    const int ly = threadIdx.x % N, j = threadIdx.x / N;
    cpx<T> va[2][R1], vb[2][R2];
    if (j < R2)
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1)
#pragma unroll
        for (int s = 0; s < 2; ++s) va[s][j1] = P[s * SP + ly * PITCH + j + R2 * j1];
    F::forward(va, vb, P + ly * PITCH, SP, 1, j, tw);
    if (j < R1)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2)
#pragma unroll
        for (int s = 0; s < 2; ++s) P[s * SP + ly * PITCH + j + R1 * k2] = vb[s][k2];
  }
  __syncthreads();
  {  // y lines, in place (column lx)
    const int lx = threadIdx.x % N, j = threadIdx.x / N;
    cpx<T> va[2][R1], vb[2][R2];
    if (j < R2)
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1)
#pragma unroll
        for (int s = 0; s < 2; ++s) va[s][j1] = P[s * SP + (j + R2 * j1) * PITCH + lx];
    F::forward(va, vb, P + lx, SP, PITCH, j, tw);
    if (j < R1)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2)
#pragma unroll
        for (int s = 0; s < 2; ++s) P[s * SP + (j + R1 * k2) * PITCH + lx] = vb[s][k2];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * C::THREADS;
    if (i < 2 * N2) {
      const int s = i / N2, q = i - s * N2;
      out[soff + s * N3 + zoff + q] = P[s * SP + (q / N) * PITCH + q % N];
    }
  }
  __syncthreads();   // P is free again: reuse it for the reduction
  const double sum = tree_sum(r2, reinterpret_cast<double*>(P));
  if (threadIdx.x == 0) r2_part[size_t(blockIdx.y) * gridDim.x + blockIdx.x] = sum * g.dV;
}

// Damped step, last half: inverse FFTs along y and x of slice z of the
// filtered spectrum in buf, then phi = psi - result, in place.
template <typename T, int N>
__global__ void __launch_bounds__(PlaneCfg<N>::THREADS)
k_damp_inv_xy(const cpx<T>* __restrict__ psi, cpx<T>* __restrict__ buf,
              unsigned int* __restrict__ amax, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using C = PlaneCfg<N>;
  using F = LineFFTInPlace<T, N, 2>;
  constexpr int R1 = C::R1, R2 = C::R2, RT = C::RT, PITCH = C::PITCH, SP = C::SPIN;
  constexpr int N2 = N * N, N3 = N * N2;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> P[2 * SP];
  load_twiddles<T, N>(tw);
  const int zoff = blockIdx.x * N2;
  const size_t soff = size_t(blockIdx.y) * 2 * N3;
  // fixed trip counts, unrolled: each thread's loads of a loop go out together
  constexpr int NIT = (2 * N2 + C::THREADS - 1) / C::THREADS;
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * C::THREADS;
    if (i < 2 * N2) {
      const int s = i / N2, q = i - s * N2;
      P[s * SP + (q / N) * PITCH + q % N] = buf[soff + s * N3 + zoff + q];
    }
  }
  __syncthreads();
  {  // y lines (column lx): frequencies -> positions
    const int lx = threadIdx.x % N, j = threadIdx.x / N;
    cpx<T> va[2][R1], vb[2][R2];
    if (j < R1)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2)
#pragma unroll
        for (int s = 0; s < 2; ++s) vb[s][k2] = P[s * SP + (j + R1 * k2) * PITCH + lx];
    F::inverse(vb, va, P + lx, SP, PITCH, j, tw);
    if (j < R2)
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1)
#pragma unroll
        for (int s = 0; s < 2; ++s) P[s * SP + (j + R2 * j1) * PITCH + lx] = va[s][j1];
  }
  __syncthreads();
  {  // x lines (row ly; rows fastest across the lanes, as in the forward half)
    const int ly = threadIdx.x % N, j = threadIdx.x / N;
    cpx<T> va[2][R1], vb[2][R2];
    if (j < R1)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2)
#pragma unroll
        for (int s = 0; s < 2; ++s) vb[s][k2] = P[s * SP + ly * PITCH + j + R1 * k2];
    F::inverse(vb, va, P + ly * PITCH, SP, 1, j, tw);
    if (j < R2)
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1)
#pragma unroll
        for (int s = 0; s < 2; ++s) P[s * SP + ly * PITCH + j + R2 * j1] = va[s][j1];
  }
  __syncthreads();
  float am = 0.0f;
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int i = threadIdx.x + it * C::THREADS;
    if (i < 2 * N2) {
      const int s = i / N2, q = i - s * N2;
      const size_t o = soff + s * N3 + zoff + q;
      const cpx<T> t = psi[o] - P[s * SP + (q / N) * PITCH + q % N];
      buf[o] = t;
      am = fmaxf(am, cabs_max(t));
    }
  }
  if (amax != nullptr) block_amax(am, amax);
}

// ------------------------------------------------------------------ damping
// phi = psi - F^-1[ x0 F(h psi - eps psi) / (E0 + hb2m |k|^2) ], done as
// forward x, forward y, (forward z, filter, inverse z), inverse y, inverse x,
// in place in the phi buffer.  The first pass also forms ||r||^2 partials.
struct DampArgs {
  double x0, e0, hb2m;
};

// pass 0: r = h psi - eps psi, forward FFT along x, store spectrum.
template <typename T, int N>
__global__ void __launch_bounds__(LineCfg<N>::THREADS)
k_damp_fwd_x(const cpx<T>* __restrict__ psi, const cpx<T>* __restrict__ hpsi,
             const double* __restrict__ eps, cpx<T>* __restrict__ out, GridArgs g,
             double* __restrict__ r2_part, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using C = LineCfg<N>;
  using F = LineFFT<T, N, 2>;
  constexpr int YS = line_stride<T, N, 2, 0>();
  constexpr int R1 = C::R1, R2 = C::R2, N3 = N * N * N;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> Ybuf[C::LPW * YS];
  __shared__ double red[4];
  load_twiddles<T, N>(tw);
  int line, j;
  thread_role<N, 0>(threadIdx.x, line, j);
  const int L = blockIdx.x * C::LPW + line;
  int base, stride, a, b;
  line_geom<N, 0>(L, base, stride, a, b);
  const size_t soff = size_t(blockIdx.y) * 2 * N3;
  const T e = T(eps[blockIdx.y]);
  cpx<T> va[2][R1], vb[2][R2];
  double r2 = 0.0;
  if (j < R2) {
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      int r = base + (j + R2 * j1) * stride;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        cpx<T> h = hpsi[soff + s * N3 + r], p = psi[soff + s * N3 + r];
        cpx<T> res = h - e * p;
        r2 += double(res.re) * double(res.re) + double(res.im) * double(res.im);
        va[s][j1] = res;
      }
    }
  }
  F::forward(va, vb, Ybuf + line * YS, j, tw);
  if (j < R1) {
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      int r = base + (j + R1 * k2) * stride;
      out[soff + r] = vb[0][k2];
      out[soff + N3 + r] = vb[1][k2];
    }
  }
  double sum = block_sum(r2, red);
  if (threadIdx.x == 0) r2_part[size_t(blockIdx.y) * gridDim.x + blockIdx.x] = sum * g.dV;
}

// forward (INV = false) or inverse (INV = true) FFT along y, in place.
template <typename T, int N, bool INV>
__global__ void __launch_bounds__(LineCfg<N>::THREADS)
k_damp_y(cpx<T>* __restrict__ buf, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using C = LineCfg<N>;
  using F = LineFFT<T, N, 2>;
  constexpr int YS = line_stride<T, N, 2, 1>();
  constexpr int R1 = C::R1, R2 = C::R2, N3 = N * N * N;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> Ybuf[C::LPW * YS];
  load_twiddles<T, N>(tw);
  int line, j;
  thread_role<N, 1>(threadIdx.x, line, j);
  const int L = blockIdx.x * C::LPW + line;
  int base, stride, a, b;
  line_geom<N, 1>(L, base, stride, a, b);
  cpx<T>* p = buf + size_t(blockIdx.y) * 2 * N3;
  cpx<T> va[2][R1], vb[2][R2];
  cpx<T>* Y = Ybuf + line * YS;
  if (!INV) {
    if (j < R2)
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1)
#pragma unroll
        for (int s = 0; s < 2; ++s) va[s][j1] = p[s * N3 + base + (j + R2 * j1) * stride];
    F::forward(va, vb, Y, j, tw);
    if (j < R1)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2)
#pragma unroll
        for (int s = 0; s < 2; ++s) p[s * N3 + base + (j + R1 * k2) * stride] = vb[s][k2];
  } else {
    if (j < R1)
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2)
#pragma unroll
        for (int s = 0; s < 2; ++s) vb[s][k2] = p[s * N3 + base + (j + R1 * k2) * stride];
    F::inverse(vb, va, Y, j, tw);
    if (j < R2)
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1)
#pragma unroll
        for (int s = 0; s < 2; ++s) p[s * N3 + base + (j + R2 * j1) * stride] = va[s][j1];
  }
}

// forward FFT along z, multiply by x0 / (E0 + hb2m |k|^2), inverse along z.
// The line's x and y indices are frequency indices at this point.
//   MODE 0: plain damping.
//   MODE 1: read only: add the state's spectral power per |k| shell,
//           sum |F r(k)|^2 over both spinor components, to pow[state][shell].
//   MODE 2: damping times gain[state][shell(k)] (learned preconditioner, or
//           one-hot rows that restrict the step to one shell).
template <typename T, int N, int MODE>
__global__ void __launch_bounds__(LineCfg<N>::THREADS)
k_damp_z(cpx<T>* __restrict__ buf, GridArgs g, DampArgs d, const float* __restrict__ gain,
         double* __restrict__ pow, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using C = LineCfg<N>;
  using F = LineFFT<T, N, 2>;
  constexpr int YS = line_stride<T, N, 2, 2>();
  constexpr int R1 = C::R1, R2 = C::R2, N3 = N * N * N;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> Ybuf[C::LPW * YS];
  __shared__ double spow[PC_SHELLS];
  load_twiddles<T, N>(tw);
  if (MODE == 1 && threadIdx.x < PC_SHELLS) spow[threadIdx.x] = 0.0;
  int line, j;
  thread_role<N, 2>(threadIdx.x, line, j);
  const int L = blockIdx.x * C::LPW + line;
  int base, stride, a, b;
  line_geom<N, 2>(L, base, stride, a, b);
  cpx<T>* p = buf + size_t(blockIdx.y) * 2 * N3;
  cpx<T>* Y = Ybuf + line * YS;
  cpx<T> va[2][R1], vb[2][R2];
  if (j < R2)
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1)
#pragma unroll
      for (int s = 0; s < 2; ++s) va[s][j1] = p[s * N3 + base + (j + R2 * j1) * stride];
  F::forward(va, vb, Y, j, tw);
  double lpow[PC_SHELLS];
  if (MODE == 1)
#pragma unroll
    for (int s = 0; s < PC_SHELLS; ++s) lpow[s] = 0.0;
  if (j < R1) {
    const int ia = a < N / 2 ? a : a - N, ib = b < N / 2 ? b : b - N;
    double kx = g.kunit * double(ia) + g.tw[0];
    double ky = g.kunit * double(ib) + g.tw[1];
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      int f = j + R1 * k2;
      const int ic = f < N / 2 ? f : f - N;
      double kz = g.kunit * double(ic) + g.tw[2];
      const double kk = kx * kx + ky * ky + kz * kz;
      const int m2 = ia * ia + ib * ib + ic * ic;
      if (MODE == 1) {
        const int sh = k_shell(m2, N);
        double pw = 0.0;
#pragma unroll
        for (int s = 0; s < 2; ++s)
          pw += double(vb[s][k2].re) * double(vb[s][k2].re) + double(vb[s][k2].im) * double(vb[s][k2].im);
#pragma unroll
        for (int s = 0; s < PC_SHELLS; ++s) lpow[s] += (s == sh) ? pw : 0.0;
      } else {
        double mm = d.x0 / (d.e0 + d.hb2m * kk);
        if (MODE == 2) mm *= double(gain[size_t(blockIdx.y) * PC_SHELLS + k_shell(m2, N)]);
        const T m = T(mm);
#pragma unroll
        for (int s = 0; s < 2; ++s) vb[s][k2] = m * vb[s][k2];
      }
    }
  }
  if (MODE == 1) {
    __syncthreads();
#pragma unroll
    for (int s = 0; s < PC_SHELLS; ++s) {
      double v = lpow[s];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if ((threadIdx.x & 63) == 0) atomicAdd(&spow[s], v);
    }
    __syncthreads();
    if (threadIdx.x < PC_SHELLS)
      atomicAdd(&pow[size_t(blockIdx.y) * PC_SHELLS + threadIdx.x], spow[threadIdx.x]);
    return;
  }
  F::inverse(vb, va, Y, j, tw);
  if (j < R2)
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1)
#pragma unroll
      for (int s = 0; s < 2; ++s) p[s * N3 + base + (j + R2 * j1) * stride] = va[s][j1];
}

// inverse FFT along x and phi = psi - (damped residual), in place in buf.
template <typename T, int N>
__global__ void __launch_bounds__(LineCfg<N>::THREADS)
k_damp_inv_x(const cpx<T>* __restrict__ psi, cpx<T>* __restrict__ buf,
             unsigned int* __restrict__ amax, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using C = LineCfg<N>;
  using F = LineFFT<T, N, 2>;
  constexpr int YS = line_stride<T, N, 2, 0>();
  constexpr int R1 = C::R1, R2 = C::R2, N3 = N * N * N;
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> Ybuf[C::LPW * YS];
  load_twiddles<T, N>(tw);
  int line, j;
  thread_role<N, 0>(threadIdx.x, line, j);
  const int L = blockIdx.x * C::LPW + line;
  int base, stride, a, b;
  line_geom<N, 0>(L, base, stride, a, b);
  const size_t soff = size_t(blockIdx.y) * 2 * N3;
  cpx<T>* Y = Ybuf + line * YS;
  cpx<T> va[2][R1], vb[2][R2];
  if (j < R1)
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2)
#pragma unroll
      for (int s = 0; s < 2; ++s) vb[s][k2] = buf[soff + s * N3 + base + (j + R1 * k2) * stride];
  F::inverse(vb, va, Y, j, tw);
  float am = 0.0f;
  if (j < R2)
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        size_t r = soff + s * N3 + base + (j + R2 * j1) * stride;
        const cpx<T> t = psi[r] - va[s][j1];
        buf[r] = t;
        am = fmaxf(am, cabs_max(t));
      }
  if (amax != nullptr) block_amax(am, amax);
}

// ------------------------------------------------------------------ densities
// Pass DIR over a chunk of states accumulates, at every point, the terms of
// rho, tau, J (and the diagnostics s, j) that need d/d(DIR) psi:
//   x: rho, s_x, s_y, s_z, tau_x, j_x, J_y(x), J_z(x)          (slots 0..7)
//   y: tau_y, j_y, J_x(y), J_z(y)                              (slots 8..11)
//   z: tau_z, j_z, J_x(z), J_y(z)                              (slots 12..15)
// with J_k = sum_lm eps_klm Im(psi^dag sigma_m d_l psi).  Partial sums per
// state chunk go to part[chunk][slot][point] and are reduced in fixed order.
template <typename T, int N, int DIR>
__global__ void __launch_bounds__(LineCfg<N>::THREADS)
k_dens_pass(DensGroups grp, int nstate, int chunk, GridArgs g, double* __restrict__ part, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using C = LineCfg<N>;
  using F = LineFFT<T, N, 2>;
  constexpr int YS = line_stride<T, N, 2, DIR>();
  constexpr int R1 = C::R1, R2 = C::R2, N3 = N * N * N;
  constexpr int NS = DIR == 0 ? 8 : 4;
  constexpr int SLOT0 = DIR == 0 ? 0 : (DIR == 1 ? 8 : 12);
  __shared__ cpx<T> tw[N];
  __shared__ cpx<T> Ybuf[C::LPW * YS];
  load_twiddles<T, N>(tw);
  int line, j;
  thread_role<N, DIR>(threadIdx.x, line, j);
  const int L = blockIdx.x * C::LPW + line;
  int base, stride, a, b;
  line_geom<N, DIR>(L, base, stride, a, b);
  cpx<T>* Y = Ybuf + line * YS;
  const T kunit = T(g.kunit);

  double acc[NS][R1];
#pragma unroll
  for (int q = 0; q < NS; ++q)
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) acc[q][j1] = 0.0;

  // chunks of the flat (group, state) index: every group's states in order;
  // the next state's line is loaded into registers while this one is
  // transformed
  const int s0 = blockIdx.y * chunk;
  const int s1 = min(nstate * grp.ngroup, s0 + chunk);
  auto load_line = [&](int fs, cpx<T> (&dst)[2][R1]) {
    const int t = fs / nstate, st = fs - t * nstate;
    const cpx<T>* p = reinterpret_cast<const cpx<T>*>(grp.psi[t]) + size_t(st) * 2 * N3;
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      const int r = base + (j + R2 * j1) * stride;
      dst[0][j1] = p[r];
      dst[1][j1] = p[N3 + r];
    }
  };
  cpx<T> vn[2][R1];
  if (s0 < s1 && j < R2) load_line(s0, vn);
  for (int fs = s0; fs < s1; ++fs) {
    const T kshift = T(grp.kshift[fs / nstate][DIR]);
    cpx<T> v[2][R1], d[2][R1];
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      v[0][j1] = d[0][j1] = vn[0][j1];
      v[1][j1] = d[1][j1] = vn[1][j1];
    }
    if (fs + 1 < s1 && j < R2) load_line(fs + 1, vn);
    F::deriv(d, Y, j, tw, kunit, kshift);
    if (j < R2) {
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) {
        cpx<T> u = v[0][j1], w = v[1][j1], du = d[0][j1], dw = d[1][j1];
        // psi^dag sigma d psi for the three Pauli matrices
        cpx<T> sx = conj(u) * dw + conj(w) * du;
        cpx<T> sy = mul_i(conj(w) * du - conj(u) * dw);
        cpx<T> sz = conj(u) * du - conj(w) * dw;
        double tau = double(norm2(du)) + double(norm2(dw));
        double cur = double((conj(u) * du).im) + double((conj(w) * dw).im);
        if (DIR == 0) {
          cpx<T> sxy = conj(u) * w;                 // psi^dag sigma psi pieces
          acc[0][j1] += double(norm2(u)) + double(norm2(w));
          acc[1][j1] += 2.0 * double(sxy.re);
          acc[2][j1] += 2.0 * double(sxy.im);
          acc[3][j1] += double(norm2(u)) - double(norm2(w));
          acc[4][j1] += tau;
          acc[5][j1] += cur;
          acc[6][j1] -= double(sz.im);             // J_y += eps_yxz Im(sz) = -Im
          acc[7][j1] += double(sy.im);             // J_z += eps_zxy Im(sy) = +Im
        } else if (DIR == 1) {
          acc[0][j1] += tau;
          acc[1][j1] += cur;
          acc[2][j1] += double(sz.im);             // J_x += eps_xyz Im(sz)
          acc[3][j1] -= double(sx.im);             // J_z += eps_zyx Im(sx)
        } else {
          acc[0][j1] += tau;
          acc[1][j1] += cur;
          acc[2][j1] -= double(sy.im);             // J_x += eps_xzy Im(sy)
          acc[3][j1] += double(sx.im);             // J_y += eps_yzx Im(sx)
        }
      }
    }
  }
  if (j < R2) {
    double* out = part + size_t(blockIdx.y) * 16 * N3;
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) {
      int r = base + (j + R2 * j1) * stride;
#pragma unroll
      for (int q = 0; q < NS; ++q) out[size_t(SLOT0 + q) * N3 + r] = acc[q][j1];
    }
  }
}

// rho, tau, J[3], s[3], j[3] (11 fields) from the chunk partials.
__global__ void k_dens_reduce(const double* __restrict__ part, int nchunk, int n3,
                              double* __restrict__ dens, double scale, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n3) return;
  double q[16];
  for (int k = 0; k < 16; ++k) q[k] = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    const double* p = part + size_t(c) * 16 * n3 + r;
    for (int k = 0; k < 16; ++k) q[k] += p[size_t(k) * n3];
  }
  if (scale != 1.0)
    for (int k = 0; k < 16; ++k) q[k] *= scale;
  double* o = dens;
  o[0 * n3 + r] = q[0];                       // rho
  o[1 * n3 + r] = q[4] + q[8] + q[12];        // tau
  o[2 * n3 + r] = q[10] + q[14];              // J_x
  o[3 * n3 + r] = q[6] + q[15];               // J_y
  o[4 * n3 + r] = q[7] + q[11];               // J_z
  o[5 * n3 + r] = q[1];                       // s_x
  o[6 * n3 + r] = q[2];                       // s_y
  o[7 * n3 + r] = q[3];                       // s_z
  o[8 * n3 + r] = q[5];                       // j_x
  o[9 * n3 + r] = q[9];                       // j_y
  o[10 * n3 + r] = q[13];                     // j_z
}

// ------------------------------------------------------------------ conversion
__global__ void k_c128_to_c64(const double2* __restrict__ a, float2* __restrict__ b, size_t n, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_float2(float(a[i].x), float(a[i].y));
}
__global__ void k_c64_to_c128(const float2* __restrict__ a, double2* __restrict__ b, size_t n, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = make_double2(double(a[i].x), double(a[i].y));
}

void convert_states(const void* src, int src_prec, void* dst, int dst_prec, size_t n,
                    hipStream_t st) {
  if (n == 0) return;
  const unsigned nb = unsigned((n + 255) / 256);
  if (src_prec == 0 && dst_prec == 1)
    hipLaunchKernelGGL(k_c128_to_c64, dim3(nb), dim3(256), 0, st, (const double2*)src, (float2*)dst, n, g_launch_gate);
  else if (src_prec == 1 && dst_prec == 0)
    hipLaunchKernelGGL(k_c64_to_c128, dim3(nb), dim3(256), 0, st, (const float2*)src, (double2*)dst, n, g_launch_gate);
  else
    hipMemcpyAsync(dst, src, n * (src_prec == 0 ? 16 : 8), hipMemcpyDeviceToDevice, st);
}

// ------------------------------------------------------------------ launchers
template <int N> static int ntiles() { return N * N / LineCfg<N>::LPW; }

// Pencil counts the h passes can run with: half, default and double the
// default lines per workgroup, where they tile the plane, fit 1024 threads
// and (double precision, double lines) the LDS.
template <int N> static constexpr bool lines_ok(int lp, int bytes_per_cpx) {
  return lp > 0 && (N * N) % lp == 0 && LineCfg<N>::RT * lp <= 1024 &&
         lp * (2 * Fact<N>::R1 * (Fact<N>::R2 + 1) + 1) * bytes_per_cpx <= 96 * 1024;
}

template <typename T, int N, int LP>
static void launch_h_lp(const void* psi, void* hpsi, int nstate, MeanFieldPtrs mf, GridArgs g,
                        double* eps_part, unsigned int* amax, hipStream_t st) {
  dim3 grid(N * N / LineCfg<N, LP>::LPW, nstate), block(LineCfg<N, LP>::THREADS);
  auto p = reinterpret_cast<const cpx<T>*>(psi);
  auto h = reinterpret_cast<cpx<T>*>(hpsi);
  hipLaunchKernelGGL((k_h_pass<T, N, 0, true, false, LP>), grid, block, 0, st, p, h, mf, g, nullptr,
                     nullptr, g_launch_gate);
  hipLaunchKernelGGL((k_h_pass<T, N, 1, false, false, LP>), grid, block, 0, st, p, h, mf, g, nullptr,
                     nullptr, g_launch_gate);
  hipLaunchKernelGGL((k_h_pass<T, N, 2, false, true, LP>), grid, block, 0, st, p, h, mf, g, eps_part,
                     amax, g_launch_gate);
}

// z pass (with U psi) by line pencils, then the x and y parts on LDS slices.
template <typename T, int N>
static void launch_h_plane(const void* psi, void* hpsi, int nstate, MeanFieldPtrs mf, GridArgs g,
                           double* eps_part, unsigned int* amax, hipStream_t st) {
  constexpr int D = LineCfg<N>::LPW;
  auto p = reinterpret_cast<const cpx<T>*>(psi);
  auto h = reinterpret_cast<cpx<T>*>(hpsi);
  hipLaunchKernelGGL((k_h_pass<T, N, 2, true, false, D>), dim3(N * N / D, nstate),
                     dim3(LineCfg<N>::THREADS), 0, st, p, h, mf, g, nullptr, nullptr, g_launch_gate);
  hipLaunchKernelGGL((k_h_plane<T, N>), dim3(N, nstate), dim3(PlaneCfg<N>::THREADS), 0, st, p, h,
                     mf, g, eps_part, amax, g_launch_gate);
}

// lines: 0 = default, H_PLANE = x and y on LDS slices, else pencils per
// workgroup of the three line passes (one of h_pass_lines).  Returns the
// eps partials (workgroups) per state, or 0 if lines is not supported.
template <typename T, int N>
static int launch_apply_h(const void* psi, void* hpsi, int nstate, MeanFieldPtrs mf, GridArgs g,
                          double* eps_part, int lines, unsigned int* amax, hipStream_t st) {
  constexpr int D = LineCfg<N>::LPW;
  constexpr int H = (D / 2 > 0 && lines_ok<N>(D / 2, sizeof(cpx<T>))) ? D / 2 : D;
  constexpr int W = lines_ok<N>(2 * D, sizeof(cpx<T>)) ? 2 * D : D;
  constexpr bool PL = plane_fits<T, N>();
  if (lines == 0) lines = plane_default<T, N>() ? H_PLANE : D;
  if (lines == H_PLANE) {
    if constexpr (PL) {
      launch_h_plane<T, N>(psi, hpsi, nstate, mf, g, eps_part, amax, st);
      return N;
    }
    return 0;
  }
  if (lines == D) { launch_h_lp<T, N, D>(psi, hpsi, nstate, mf, g, eps_part, amax, st); return N * N / D; }
  if (lines == H) { launch_h_lp<T, N, H>(psi, hpsi, nstate, mf, g, eps_part, amax, st); return N * N / H; }
  if (lines == W) { launch_h_lp<T, N, W>(psi, hpsi, nstate, mf, g, eps_part, amax, st); return N * N / W; }
  return 0;
}

// Candidates of the tuner: the slice variant (where it fits), then half,
// default and double pencils (deduplicated).  Returns the count.
template <typename T, int N> static int lines_list(int* out) {
  constexpr int D = LineCfg<N>::LPW;
  int k = 0;
  if (plane_fits<T, N>()) out[k++] = H_PLANE;
  const int c[3] = {(D / 2 > 0 && lines_ok<N>(D / 2, sizeof(cpx<T>))) ? D / 2 : D, D,
                    lines_ok<N>(2 * D, sizeof(cpx<T>)) ? 2 * D : D};
  for (int i = 0; i < 3; ++i) {
    bool dup = false;
    for (int m = 0; m < k; ++m) dup = dup || out[m] == c[i];
    if (!dup) out[k++] = c[i];
  }
  return k;
}

template <typename T, int N> static int lines_default() {
  return plane_default<T, N>() ? H_PLANE : LineCfg<N>::LPW;
}

int grid_ntiles(int n) {
  int r = 0;
  SKY_DISPATCH_N(n, r = std::max(2 * ntiles<NN>(), NN));
  return r;   // room for the h passes at half the default pencils, or one per slice
}

int h_pass_lines(int n, int prec, int* out) {
  int k = 0;
  if (prec == 0) SKY_DISPATCH_N(n, k = (lines_list<double, NN>(out)))
  else SKY_DISPATCH_N(n, k = (lines_list<float, NN>(out)))
  return k;
}

int damp_slices_available(int n, int prec) {
  int v = 0;
  if (prec == 0) SKY_DISPATCH_N(n, v = (damp_slices_fit<double, NN>() ? 1 : 0))
  else SKY_DISPATCH_N(n, v = (damp_slices_fit<float, NN>() ? 1 : 0))
  return v;
}

int h_pass_default(int n, int prec) {
  int v = 0;
  if (prec == 0) SKY_DISPATCH_N(n, v = (lines_default<double, NN>()))
  else SKY_DISPATCH_N(n, v = (lines_default<float, NN>()))
  return v;
}

int apply_h(int n, int prec, const void* psi, void* hpsi, int nstate, MeanFieldPtrs mf,
            GridArgs g, double* eps_part, double* eps, hipStream_t st, int lines,
            unsigned int* amax) {
  if (nstate <= 0) return 1;
  int nt = 0;
  if (prec == 0) SKY_DISPATCH_N(n, nt = (launch_apply_h<double, NN>(psi, hpsi, nstate, mf, g, eps_part, lines, amax, st)))
  else SKY_DISPATCH_N(n, nt = (launch_apply_h<float, NN>(psi, hpsi, nstate, mf, g, eps_part, lines, amax, st)))
  if (nt == 0) return 0;
  if (eps_part && eps)
    hipLaunchKernelGGL(k_sum_partials, dim3((nstate + 127) / 128), dim3(128), 0, st,
                       (const double*)eps_part, nt, nstate, eps, g_launch_gate);
  return 1;
}

// stage 0: the whole step; 1: residual, forward x and y and (with shell_pow)
// the shell powers, leaving the partial spectrum in phi; 2: the z filter
// (with gain) and the inverse passes, continuing from stage 1.
template <typename T, int N>
static void launch_damp(const void* psi, const void* hpsi, const double* eps, void* phi,
                        int nstate, GridArgs g, DampArgs d, double* r2_part, const float* gain,
                        double* shell_pow, int stage, int xy, unsigned int* amax, hipStream_t st) {
  dim3 grid(ntiles<N>(), nstate), block(LineCfg<N>::THREADS);
  dim3 pgrid(N, nstate), pblock(PlaneCfg<N>::THREADS);
  auto p = reinterpret_cast<const cpx<T>*>(psi);
  auto h = reinterpret_cast<const cpx<T>*>(hpsi);
  auto o = reinterpret_cast<cpx<T>*>(phi);
  const bool pl = damp_slices_fit<T, N>() && (xy < 0 ? damp_slice_default<T, N>() : xy != 0);
  if (stage != 2) {
    if (pl) {
      if constexpr (damp_slices_fit<T, N>())
        hipLaunchKernelGGL((k_damp_fwd_xy<T, N>), pgrid, pblock, 0, st, p, h, eps, o, g, r2_part, g_launch_gate);
    } else {
      hipLaunchKernelGGL((k_damp_fwd_x<T, N>), grid, block, 0, st, p, h, eps, o, g, r2_part, g_launch_gate);
      hipLaunchKernelGGL((k_damp_y<T, N, false>), grid, block, 0, st, o, g_launch_gate);
    }
    if (shell_pow)
      hipLaunchKernelGGL((k_damp_z<T, N, 1>), grid, block, 0, st, o, g, d, nullptr, shell_pow, g_launch_gate);
  }
  if (stage == 1) return;
  if (gain)
    hipLaunchKernelGGL((k_damp_z<T, N, 2>), grid, block, 0, st, o, g, d, gain, nullptr, g_launch_gate);
  else
    hipLaunchKernelGGL((k_damp_z<T, N, 0>), grid, block, 0, st, o, g, d, nullptr, nullptr, g_launch_gate);
  if (pl) {
    if constexpr (damp_slices_fit<T, N>())
      hipLaunchKernelGGL((k_damp_inv_xy<T, N>), pgrid, pblock, 0, st, p, o, amax, g_launch_gate);
  } else {
    hipLaunchKernelGGL((k_damp_y<T, N, true>), grid, block, 0, st, o, g_launch_gate);
    hipLaunchKernelGGL((k_damp_inv_x<T, N>), grid, block, 0, st, p, o, amax, g_launch_gate);
  }
}

void damped_step(int n, int prec, const void* psi, const void* hpsi, const double* eps,
                 void* phi, int nstate, GridArgs g, double x0, double e0, double hb2m,
                 double* r2_part, double* r2, hipStream_t st, const float* gain,
                 double* shell_pow, int stage, int xy, unsigned int* amax) {
  if (nstate <= 0) return;
  DampArgs d{x0, e0, hb2m};
  if (prec == 0) SKY_DISPATCH_N(n, launch_damp<double, NN>(psi, hpsi, eps, phi, nstate, g, d, r2_part, gain, shell_pow, stage, xy, amax, st))
  else SKY_DISPATCH_N(n, launch_damp<float, NN>(psi, hpsi, eps, phi, nstate, g, d, r2_part, gain, shell_pow, stage, xy, amax, st))
  if (stage == 2) return;
  int nt = 0;
  if (prec == 0)
    SKY_DISPATCH_N(n, nt = (damp_slices_fit<double, NN>() && (xy < 0 ? damp_slice_default<double, NN>() : xy != 0)) ? NN : ntiles<NN>())
  else
    SKY_DISPATCH_N(n, nt = (damp_slices_fit<float, NN>() && (xy < 0 ? damp_slice_default<float, NN>() : xy != 0)) ? NN : ntiles<NN>())
  if (r2)
    hipLaunchKernelGGL(k_sum_partials, dim3((nstate + 127) / 128), dim3(128), 0, st,
                       (const double*)r2_part, nt, nstate, r2, g_launch_gate);
}

template <typename T, int N>
static void launch_dens(const DensGroups& grp, int nstate, int chunk, int nchunk, GridArgs g,
                        double* part, hipStream_t st) {
  dim3 grid(ntiles<N>(), nchunk), block(LineCfg<N>::THREADS);
  hipLaunchKernelGGL((k_dens_pass<T, N, 0>), grid, block, 0, st, grp, nstate, chunk, g, part, g_launch_gate);
  hipLaunchKernelGGL((k_dens_pass<T, N, 1>), grid, block, 0, st, grp, nstate, chunk, g, part, g_launch_gate);
  hipLaunchKernelGGL((k_dens_pass<T, N, 2>), grid, block, 0, st, grp, nstate, chunk, g, part, g_launch_gate);
}

int densities(int n, int prec, const void* const* psi, const GridArgs* g, int ngroup,
              int nstate, int nchunk_max, double* part, double* dens, hipStream_t st) {
  const int n3 = n * n * n;
  if (ngroup < 0 || ngroup > DENS_MAX_GROUPS || nchunk_max < 1) return 0;
  if (nstate <= 0 || ngroup == 0) {
    zero(dens, size_t(11) * n3, st);
    return 1;
  }
  // one launch per pass over all groups (twists): the flat (group, state)
  // index is cut into at most nchunk_max chunks of consecutive states
  DensGroups grp{};
  grp.ngroup = ngroup;
  for (int t = 0; t < ngroup; ++t) {
    grp.psi[t] = psi[t];
    for (int a = 0; a < 3; ++a) grp.kshift[t][a] = g[t].tw[a];
  }
  const int total = ngroup * nstate;
  const int chunk = (total + nchunk_max - 1) / nchunk_max;
  const int nchunk = (total + chunk - 1) / chunk;
  if (prec == 0) SKY_DISPATCH_N(n, launch_dens<double, NN>(grp, nstate, chunk, nchunk, g[0], part, st))
  else SKY_DISPATCH_N(n, launch_dens<float, NN>(grp, nstate, chunk, nchunk, g[0], part, st))
  hipLaunchKernelGGL(k_dens_reduce, dim3((n3 + 255) / 256), dim3(256), 0, st,
                     (const double*)part, nchunk, n3, dens, 1.0 / ngroup, g_launch_gate);
  return 1;
}

}  // namespace sky
