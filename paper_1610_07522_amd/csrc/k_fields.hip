// Mean field of the Skyrme functional from the local densities, the Coulomb
// potential solved in momentum space, and the total energy.
//
// Sec. 2.2: h = kinetic + Skyrme mean field (Eq. Skyrme) + Coulomb, with the
// Coulomb problem solved by FFTs; Fig. 1 step 4b.  The fields are small
// (a few n^3 arrays), so each line transform here is one thread doing a
// direct DFT of its line; the cost is negligible next to the per-state work.
#include "sky_kernels.h"

namespace sky {

namespace {
constexpr int FL_THREADS = 32;  // lines per workgroup in the field kernels
constexpr int E_THREADS = 256;  // threads per energy-reduction block
constexpr int NTERM = 7;        // energy terms

__device__ inline int line_base(int L, int n, int dir, int& a, int& b, int& stride) {
  a = L % n;
  b = L / n;
  if (dir == 0) { stride = 1; return b * n * n + a * n; }
  if (dir == 1) { stride = n; return b * n * n + a; }
  stride = n * n;
  return b * n + a;
}

__device__ inline double kval(int f, int n, double kunit) {
  return kunit * double(f < n / 2 ? f : f - n);
}

// Real field -> real field spectral op along `dir`:
//   kind 0: multiply by i k (Nyquist zeroed)      -> first derivative
//   kind 1: multiply by -k^2 (Nyquist kept)        -> second derivative
// dst = (accumulate ? dst : 0) + Re F^-1[m(k) F src].
__global__ void k_field_line(const double* __restrict__ src, double* __restrict__ dst, int n,
                             int dir, int kind, double kunit, int accumulate) {
  extern __shared__ double sh[];
  const int L = blockIdx.x * FL_THREADS + threadIdx.x;
  double* twr = sh;                      // n cos values
  double* twi = sh + n;                  // n sin values (forward sign)
  double* Xr = sh + 2 * n + threadIdx.x * 2 * n;
  double* Xi = Xr + n;
  for (int m = threadIdx.x; m < n; m += blockDim.x) {
    double s, c;
    sincospi(-2.0 * double(m) / double(n), &s, &c);
    twr[m] = c;
    twi[m] = s;
  }
  __syncthreads();
  if (L >= n * n) return;
  int a, b, stride;
  int base = line_base(L, n, dir, a, b, stride);
  for (int k = 0; k < n; ++k) {          // forward DFT of a real line
    double sr = 0.0, si = 0.0;
    for (int x = 0; x < n; ++x) {
      int m = (x * k) % n;
      double v = src[base + x * stride];
      sr += v * twr[m];
      si += v * twi[m];
    }
    double kk = kval(k, n, kunit);
    double mr, mi;                       // multiplier m(k) = mr + i mi
    if (kind == 0) { mr = 0.0; mi = (k == n / 2) ? 0.0 : kk; }
    else { mr = -kk * kk; mi = 0.0; }
    Xr[k] = sr * mr - si * mi;
    Xi[k] = sr * mi + si * mr;
  }
  const double inv_n = 1.0 / double(n);
  for (int x = 0; x < n; ++x) {          // real part of the inverse DFT
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
      int m = (x * k) % n;
      s += Xr[k] * twr[m] + Xi[k] * twi[m];  // Re[X conj(w)]
    }
    s *= inv_n;
    double* o = dst + base + x * stride;
    *o = accumulate ? *o + s : s;
  }
}

// In-place complex DFT of every line along `dir` (forward or inverse, the
// inverse carrying 1/n).
__global__ void k_field_fft(double2* __restrict__ buf, int n, int dir, int inverse) {
  extern __shared__ double sh[];
  const int L = blockIdx.x * FL_THREADS + threadIdx.x;
  double* twr = sh;
  double* twi = sh + n;
  double* Xr = sh + 2 * n + threadIdx.x * 2 * n;
  double* Xi = Xr + n;
  for (int m = threadIdx.x; m < n; m += blockDim.x) {
    double s, c;
    sincospi(-2.0 * double(m) / double(n), &s, &c);
    twr[m] = c;
    twi[m] = inverse ? -s : s;
  }
  __syncthreads();
  if (L >= n * n) return;
  int a, b, stride;
  int base = line_base(L, n, dir, a, b, stride);
  for (int k = 0; k < n; ++k) {
    double sr = 0.0, si = 0.0;
    for (int x = 0; x < n; ++x) {
      int m = (x * k) % n;
      double2 v = buf[base + x * stride];
      sr += v.x * twr[m] - v.y * twi[m];
      si += v.x * twi[m] + v.y * twr[m];
    }
    Xr[k] = sr;
    Xi[k] = si;
  }
  const double sc = inverse ? 1.0 / double(n) : 1.0;
  for (int k = 0; k < n; ++k) buf[base + k * stride] = make_double2(sc * Xr[k], sc * Xi[k]);
}

__global__ void k_real_to_cpx(const double* __restrict__ src, double2* __restrict__ dst, int n3) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n3) dst[r] = make_double2(src[r], 0.0);
}

// V(k) = 4 pi e2 rho(k) / |k|^2, zero at k = 0.
__global__ void k_coulomb_mult(double2* __restrict__ buf, int n, double kunit, double e2) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n * n * n) return;
  int x = r % n, y = (r / n) % n, z = r / (n * n);
  double kx = kval(x, n, kunit), ky = kval(y, n, kunit), kz = kval(z, n, kunit);
  double k2 = kx * kx + ky * ky + kz * kz;
  double f = (r == 0) ? 0.0 : 4.0 * M_PI * e2 / k2;
  double2 v = buf[r];
  buf[r] = make_double2(f * v.x, f * v.y);
}

__global__ void k_cpx_real_part(const double2* __restrict__ src, double* __restrict__ dst, int n3) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n3) dst[r] = src[r].x;
}

// U, B, W of both species and the per-block energy partials.
// dens: [rho, tau, Jx, Jy, Jz, ...]; derived: [lap rho, drho x/y/z, div J].
__global__ void k_mean_field(Skyrme sk, int n3, double dV, const double* __restrict__ dn,
                             const double* __restrict__ dp, const double* __restrict__ gn,
                             const double* __restrict__ gp, const double* __restrict__ vc,
                             double* __restrict__ mn, double* __restrict__ mp,
                             double* __restrict__ epart) {
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

__global__ void k_energy_final(const double* __restrict__ epart, int nblk, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double tot = 0.0;
  for (int t = 0; t < NTERM; ++t) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += epart[b * NTERM + t];
    out[t] = s;
    tot += s;
  }
  out[NTERM] = tot;
}

void field_op(const double* src, double* dst, int n, int dir, int kind, double kunit,
              int accumulate, hipStream_t st) {
  size_t shm = sizeof(double) * (2 * n + FL_THREADS * 2 * n);
  hipLaunchKernelGGL(k_field_line, dim3((n * n + FL_THREADS - 1) / FL_THREADS),
                     dim3(FL_THREADS), shm, st, src, dst, n, dir, kind, kunit, accumulate);
}

void field_fft(double2* buf, int n, int dir, int inverse, hipStream_t st) {
  size_t shm = sizeof(double) * (2 * n + FL_THREADS * 2 * n);
  hipLaunchKernelGGL(k_field_fft, dim3((n * n + FL_THREADS - 1) / FL_THREADS), dim3(FL_THREADS),
                     shm, st, buf, n, dir, inverse);
}
}  // namespace

int energy_nblocks(int n) { return (n * n * n + E_THREADS - 1) / E_THREADS; }

void mean_field(int n, GridArgs g, const Skyrme& sk, const double* dens_n, const double* dens_p,
                double* der_n, double* der_p, double* mf_n, double* mf_p, double* vc,
                void* scratch, double* epart, double* energy, hipStream_t st) {
  const int n3 = n * n * n;
  const double* dens[2] = {dens_n, dens_p};
  double* der[2] = {der_n, der_p};
  for (int q = 0; q < 2; ++q) {
    const double* rho = dens[q];
    const double* J = dens[q] + 2 * n3;
    double* o = der[q];
    // Laplacian: sum over axes of the -k^2 multiplier (Nyquist kept)
    for (int m = 0; m < 3; ++m) field_op(rho, o, n, m, 1, g.kunit, m > 0, st);
    // gradient (Nyquist zeroed)
    for (int m = 0; m < 3; ++m) field_op(rho, o + (1 + m) * n3, n, m, 0, g.kunit, 0, st);
    // divergence of J
    for (int m = 0; m < 3; ++m) field_op(J + m * n3, o + 4 * n3, n, m, 0, g.kunit, m > 0, st);
  }
  const double* vcp = nullptr;
  if (sk.e2 != 0.0) {
    double2* buf = reinterpret_cast<double2*>(scratch);
    hipLaunchKernelGGL(k_real_to_cpx, dim3((n3 + 255) / 256), dim3(256), 0, st, dens_p, buf, n3);
    for (int m = 0; m < 3; ++m) field_fft(buf, n, m, 0, st);
    hipLaunchKernelGGL(k_coulomb_mult, dim3((n3 + 255) / 256), dim3(256), 0, st, buf, n,
                       g.kunit, sk.e2);
    for (int m = 2; m >= 0; --m) field_fft(buf, n, m, 1, st);
    hipLaunchKernelGGL(k_cpx_real_part, dim3((n3 + 255) / 256), dim3(256), 0, st,
                       (const double2*)buf, vc, n3);
    vcp = vc;
  } else {
    zero(vc, n3, st);
  }
  const int nblk = energy_nblocks(n);
  hipLaunchKernelGGL(k_mean_field, dim3(nblk), dim3(E_THREADS), 0, st, sk, n3, g.dV, dens_n,
                     dens_p, (const double*)der_n, (const double*)der_p, vcp, mf_n, mf_p, epart);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, st, (const double*)epart, nblk,
                     energy);
}

}  // namespace sky
