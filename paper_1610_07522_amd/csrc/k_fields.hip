// Mean field of the Skyrme functional from the local densities, the Coulomb
// potential solved in momentum space, and the total energy.
//
// Sec. 2.2: h = kinetic + Skyrme mean field (Eq. Skyrme) + Coulomb, with the
// Coulomb problem solved by FFTs; Fig. 1 step 4b.  The fields are small
// (a few n^3 arrays).  A spectral first derivative (Nyquist zeroed) or
// second derivative of a real field along one axis is a real circulant on
// each grid line, so all of them are n-tap circular convolutions with taps
// computed once per call; the Coulomb transform is a direct DFT pass per
// axis with one thread per output element.
#include "sky_kernels.h"

namespace sky {

namespace {
constexpr int E_THREADS = 256;  // threads per energy-reduction block
constexpr int NTERM = 7;        // energy terms

__device__ inline double kval(int f, int n, double kunit) {
  return kunit * double(f < n / 2 ? f : f - n);
}

// Taps of the line operators and the DFT twiddles, tab[4n]:
//   c0[d] = (1/n) sum_k i k e^{2 pi i k d / n}   (Nyquist k zeroed): first derivative
//   c1[d] = (1/n) sum_k -k^2 e^{2 pi i k d / n}  (Nyquist kept): second derivative
// (both real: the multipliers are odd / even in k), tw[d] = e^{-2 pi i d / n}.
// out[x] = sum_x' src[x'] c[(x - x') mod n] along a line.
__global__ void k_field_tables(double* __restrict__ tab, int n, double kunit, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int d = threadIdx.x;
  if (d >= n) return;
  double a0 = 0.0, a1 = 0.0;
  for (int k = 0; k < n; ++k) {
    double sn, cs;
    sincospi(2.0 * double((k * d) % n) / double(n), &sn, &cs);
    const double kk = kval(k, n, kunit);
    if (2 * k != n) a0 -= kk * sn;
    a1 -= kk * kk * cs;
  }
  tab[d] = a0 / double(n);
  tab[n + d] = a1 / double(n);
  double sn, cs;
  sincospi(-2.0 * double(d) / double(n), &sn, &cs);
  tab[2 * n + d] = cs;
  tab[3 * n + d] = sn;
}

// o = [lap rho, d rho/dx, d rho/dy, d rho/dz, div J] at every point.
__global__ void __launch_bounds__(256)
k_field_derivs(const double* __restrict__ rho, const double* __restrict__ J, double* __restrict__ o,
               int n, const double* __restrict__ tab, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double c0[64], c1[64];
  if (threadIdx.x < n) {
    c0[threadIdx.x] = tab[threadIdx.x];
    c1[threadIdx.x] = tab[n + threadIdx.x];
  }
  __syncthreads();
  const int n2 = n * n, n3 = n2 * n;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n3) return;
  const int x = p % n, y = (p / n) % n, z = p / n2;
  const double* Jx = J;
  const double* Jy = J + n3;
  const double* Jz = J + 2 * n3;
  double lap = 0.0, gx = 0.0, gy = 0.0, gz = 0.0, dj = 0.0;
  const int bx = z * n2 + y * n, by = z * n2 + x, bz = y * n + x;
  for (int j = 0; j < n; ++j) {
    const int dx = x - j < 0 ? x - j + n : x - j;
    const int dy = y - j < 0 ? y - j + n : y - j;
    const int dz = z - j < 0 ? z - j + n : z - j;
    const double rx = rho[bx + j], ry = rho[by + j * n], rz = rho[bz + j * n2];
    lap += c1[dx] * rx + c1[dy] * ry + c1[dz] * rz;
    gx += c0[dx] * rx;
    gy += c0[dy] * ry;
    gz += c0[dz] * rz;
    dj += c0[dx] * Jx[bx + j] + c0[dy] * Jy[by + j * n] + c0[dz] * Jz[bz + j * n2];
  }
  o[p] = lap;
  o[n3 + p] = gx;
  o[2 * n3 + p] = gy;
  o[3 * n3 + p] = gz;
  o[4 * n3 + p] = dj;
}

// One axis of a 3D DFT: dst[.., k, ..] = s * sum_j src[.., j, ..] w^{+-k j}
// (forward e^{-2 pi i k j / n}; inverse the conjugate and s = 1/n).
__global__ void __launch_bounds__(256)
k_dft_pass(const double2* __restrict__ src, double2* __restrict__ dst, int n, int dir, int inverse,
           const double* __restrict__ tab, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double twr[64], twi[64];
  if (threadIdx.x < n) {
    twr[threadIdx.x] = tab[2 * n + threadIdx.x];
    twi[threadIdx.x] = inverse ? -tab[3 * n + threadIdx.x] : tab[3 * n + threadIdx.x];
  }
  __syncthreads();
  const int n2 = n * n, n3 = n2 * n;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n3) return;
  const int x = p % n, y = (p / n) % n, z = p / n2;
  int k, base, stride;
  if (dir == 0) { k = x; base = z * n2 + y * n; stride = 1; }
  else if (dir == 1) { k = y; base = z * n2 + x; stride = n; }
  else { k = z; base = y * n + x; stride = n2; }
  double sr = 0.0, si = 0.0;
  int t = 0;   // (k * j) mod n
  for (int j = 0; j < n; ++j) {
    const double2 v = src[base + j * stride];
    sr += v.x * twr[t] - v.y * twi[t];
    si += v.x * twi[t] + v.y * twr[t];
    t += k;
    if (t >= n) t -= n;
  }
  const double sc = inverse ? 1.0 / double(n) : 1.0;
  dst[p] = make_double2(sc * sr, sc * si);
}

__global__ void k_real_to_cpx(const double* __restrict__ src, double2* __restrict__ dst, int n3, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n3) dst[r] = make_double2(src[r], 0.0);
}

// V(k) = 4 pi e2 rho(k) / |k|^2, zero at k = 0.
__global__ void k_coulomb_mult(double2* __restrict__ buf, int n, double kunit, double e2, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n * n * n) return;
  int x = r % n, y = (r / n) % n, z = r / (n * n);
  double kx = kval(x, n, kunit), ky = kval(y, n, kunit), kz = kval(z, n, kunit);
  double k2 = kx * kx + ky * ky + kz * kz;
  double f = (r == 0) ? 0.0 : 4.0 * M_PI * e2 / k2;
  double2 v = buf[r];
  buf[r] = make_double2(f * v.x, f * v.y);
}

__global__ void k_cpx_real_part(const double2* __restrict__ src, double* __restrict__ dst, int n3, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n3) dst[r] = src[r].x;
}

// U, B, W of both species and the per-block energy partials.
// dens: [rho, tau, Jx, Jy, Jz, ...]; derived: [lap rho, drho x/y/z, div J].
__global__ void k_mean_field(Skyrme sk, int n3, double dV, const double* __restrict__ dn,
                             const double* __restrict__ dp, const double* __restrict__ gn,
                             const double* __restrict__ gp, const double* __restrict__ vc,
                             double* __restrict__ mn, double* __restrict__ mp,
                             double* __restrict__ epart, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double red[NTERM][E_THREADS / 64];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  double e[NTERM] = {0, 0, 0, 0, 0, 0, 0};
  if (r < n3) {
    const double rn = dn[r], rp = dp[r], tn = dn[n3 + r], tp = dp[n3 + r];
    const double ln = gn[r], lp = gp[r], djn = gn[4 * n3 + r], djp = gp[4 * n3 + r];
    const double rho = rn + rp, tau = tn + tp, lap = ln + lp, divJ = djn + djp;
    const double vcr = vc ? vc[r] : 0.0;
    const double rs = fmax(rho, 1e-30);
    const double ra = pow(rs, sk.alpha);
    const double sq = rn * rn + rp * rp;
    const double common = sk.b0 * rho + sk.b1 * tau - sk.b2 * lap - sk.b4 * divJ +
                          sk.b3 / 3.0 * (sk.alpha + 2.0) * ra * rs -
                          sk.b3p / 3.0 * sk.alpha * ra * (sq / rs);
    for (int q = 0; q < 2; ++q) {
      const double rq = q ? rp : rn, tq = q ? tp : tn, lq = q ? lp : ln, dq = q ? djp : djn;
      const double* gq = q ? gp : gn;
      double* m = q ? mp : mn;
      double U = common - sk.b0p * rq - sk.b1p * tq + sk.b2p * lq - sk.b4p * dq -
                 sk.b3p / 3.0 * 2.0 * ra * rq;
      if (q) U += vcr;
      m[r] = U;
      m[n3 + r] = (q ? sk.hb2m_p : sk.hb2m_n) + sk.b1 * rho - sk.b1p * rq;
      for (int c = 0; c < 3; ++c) {
        const double grad = gn[(1 + c) * n3 + r] + gp[(1 + c) * n3 + r];
        m[(2 + c) * n3 + r] = sk.b4 * grad + sk.b4p * gq[(1 + c) * n3 + r];
      }
    }
    e[0] = sk.hb2m_n * tn + sk.hb2m_p * tp;
    e[1] = sk.b0 / 2.0 * rho * rho - sk.b0p / 2.0 * sq;
    e[2] = sk.b3 / 3.0 * ra * rs * rs - sk.b3p / 3.0 * ra * sq;
    e[3] = sk.b1 * rho * tau - sk.b1p * (rn * tn + rp * tp);
    e[4] = -sk.b2 / 2.0 * rho * lap + sk.b2p / 2.0 * (rn * ln + rp * lp);
    e[5] = -sk.b4 * rho * divJ - sk.b4p * (rn * djn + rp * djp);
    e[6] = 0.5 * rp * vcr;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int t = 0; t < NTERM; ++t) {
    double v = e[t];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[t][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < NTERM) {
    double s = 0.0;
    for (int w = 0; w < E_THREADS / 64; ++w) s += red[threadIdx.x][w];
    epart[blockIdx.x * NTERM + threadIdx.x] = s * dV;
  }
}

// out[t] = sum of the block partials of term t in block order (thread t;
// the loop unrolled so that the loads overlap), out[NTERM] = sum of the terms.
__global__ void k_energy_final(const double* __restrict__ epart, int nblk, double* __restrict__ out, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double term[NTERM];
  const int t = threadIdx.x;
  if (t < NTERM) {
    double s = 0.0;
#pragma unroll 8
    for (int b = 0; b < nblk; ++b) s += epart[b * NTERM + t];
    out[t] = s;
    term[t] = s;
  }
  __syncthreads();
  if (t == 0) {
    double tot = 0.0;
    for (int k = 0; k < NTERM; ++k) tot += term[k];
    out[NTERM] = tot;
  }
}

}  // namespace

int energy_nblocks(int n) { return (n * n * n + E_THREADS - 1) / E_THREADS; }

size_t mean_field_scratch_bytes(int n) {
  return 2 * sizeof(double2) * size_t(n) * n * n + 4 * sizeof(double) * size_t(n);
}

void mean_field(int n, GridArgs g, const Skyrme& sk, const double* dens_n, const double* dens_p,
                double* der_n, double* der_p, double* mf_n, double* mf_p, double* vc,
                void* scratch, double* epart, double* energy, hipStream_t st) {
  const int n3 = n * n * n;
  const double* dens[2] = {dens_n, dens_p};
  double* der[2] = {der_n, der_p};
  double2* bufA = reinterpret_cast<double2*>(scratch);
  double2* bufB = bufA + n3;
  double* tab = reinterpret_cast<double*>(bufB + n3);
  hipLaunchKernelGGL(k_field_tables, dim3(1), dim3(64), 0, st, tab, n, g.kunit, g_launch_gate);
  const unsigned nb = unsigned((n3 + 255) / 256);
  for (int q = 0; q < 2; ++q)   // lap rho (Nyquist kept), grad rho, div J (Nyquist zeroed)
    hipLaunchKernelGGL(k_field_derivs, dim3(nb), dim3(256), 0, st, dens[q], dens[q] + 2 * n3,
                       der[q], n, (const double*)tab, g_launch_gate);
  const double* vcp = nullptr;
  if (sk.e2 != 0.0) {
    hipLaunchKernelGGL(k_real_to_cpx, dim3(nb), dim3(256), 0, st, dens_p, bufA, n3, g_launch_gate);
    hipLaunchKernelGGL(k_dft_pass, dim3(nb), dim3(256), 0, st, (const double2*)bufA, bufB, n, 0, 0, (const double*)tab, g_launch_gate);
    hipLaunchKernelGGL(k_dft_pass, dim3(nb), dim3(256), 0, st, (const double2*)bufB, bufA, n, 1, 0, (const double*)tab, g_launch_gate);
    hipLaunchKernelGGL(k_dft_pass, dim3(nb), dim3(256), 0, st, (const double2*)bufA, bufB, n, 2, 0, (const double*)tab, g_launch_gate);
    hipLaunchKernelGGL(k_coulomb_mult, dim3(nb), dim3(256), 0, st, bufB, n, g.kunit, sk.e2, g_launch_gate);
    hipLaunchKernelGGL(k_dft_pass, dim3(nb), dim3(256), 0, st, (const double2*)bufB, bufA, n, 2, 1, (const double*)tab, g_launch_gate);
    hipLaunchKernelGGL(k_dft_pass, dim3(nb), dim3(256), 0, st, (const double2*)bufA, bufB, n, 1, 1, (const double*)tab, g_launch_gate);
    hipLaunchKernelGGL(k_dft_pass, dim3(nb), dim3(256), 0, st, (const double2*)bufB, bufA, n, 0, 1, (const double*)tab, g_launch_gate);
    hipLaunchKernelGGL(k_cpx_real_part, dim3(nb), dim3(256), 0, st, (const double2*)bufA, vc, n3, g_launch_gate);
    vcp = vc;
  } else {
    zero(vc, n3, st);
  }
  const int nblk = energy_nblocks(n);
  hipLaunchKernelGGL(k_mean_field, dim3(nblk), dim3(E_THREADS), 0, st, sk, n3, g.dV, dens_n,
                     dens_p, (const double*)der_n, (const double*)der_p, vcp, mf_n, mf_p, epart, g_launch_gate);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, st, (const double*)epart, nblk,
                     energy, g_launch_gate);
}

}  // namespace sky
