// Dense FP64 Hermitian linear algebra of the subspace step (Sec. 3.3.2):
// Cholesky factor of the overlap and its inverse (the orthonormalising
// transform), and a Hermitian eigensolver for the subspace Hamiltonian.
//
// The eigensolver is a blocked two-sided Jacobi method: the matrix is cut
// into 32-wide blocks, block pairs are visited in round-robin order, each
// 64x64 pair sub-matrix is diagonalised inside one workgroup (cyclic Jacobi
// in LDS), and the resulting unitaries are applied to the whole matrix and
// to the eigenvector accumulator.  Jacobi suits this step because the
// subspace Hamiltonian is nearly diagonal after the first iterations, and
// every round is fully parallel.
#include <vector>
#include <algorithm>
#include <cmath>

#include "jacobi_rot.h"
#include "mfma_f64.h"
#include "sky_kernels.h"

namespace sky {

thread_local const int* g_launch_gate = nullptr;


namespace {
using namespace jrot;
constexpr int CB = 64;    // Cholesky block
constexpr int JB = 16;    // Jacobi block (pair sub-problem = 2*JB)
constexpr int JP = 2 * JB;
constexpr int JE = JP * JP / 256;   // pair-matrix elements per thread (256 threads)
constexpr int RV = 64;              // rows of V per workgroup in the V update
// Cyclic sweeps per pair sub-problem and round.  The pair tolerance is 100x
// tighter than the global one so that the ~(n/32)^2/2 converged pair blocks
// together stay below the global off-diagonal bound.
constexpr int JACOBI_INNER = 3;

// ------------------------------------------------------------------ Cholesky
// Factor the kw x kw diagonal block at (k0, k0) in LDS and invert it:
// A[k0.., k0..] <- L_kk (lower), Dinv <- L_kk^-1 (CB x CB, lower).
__global__ void __launch_bounds__(256)
k_chol_diag(double2* __restrict__ A, int m, int k0, double2* __restrict__ Dinv, int* info,
            double piv_min, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double2 S[CB][CB + 1];
  __shared__ double2 X[CB][CB + 1];
  __shared__ int bad;
  const int kw = min(CB, m - k0);
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < CB * CB; e += blockDim.x) {
    int i = e / CB, j = e % CB;
    S[i][j] = (i < kw && j < kw) ? A[size_t(k0 + i) * m + k0 + j] : make_double2(0, 0);
    X[i][j] = make_double2(0, 0);
  }
  __syncthreads();
  for (int j = 0; j < kw; ++j) {
    if (tid == 0) {
      double d = S[j][j].x;
      if (!(d > piv_min)) { bad = 1; d = 1.0; }
      S[j][j] = make_double2(sqrt(d), 0.0);
    }
    __syncthreads();
    const double inv = 1.0 / S[j][j].x;
    for (int i = j + 1 + tid; i < kw; i += blockDim.x) S[i][j] = cscale(inv, S[i][j]);
    __syncthreads();
    // trailing update of the lower part: S[i][l] -= L[i][j] conj(L[l][j]), i >= l > j
    const int w = kw - j - 1;
    for (int e = tid; e < w * w; e += blockDim.x) {
      int i = j + 1 + e / w, l = j + 1 + e % w;
      if (l <= i) S[i][l] = csub(S[i][l], cmulc(S[i][j], S[l][j]));
    }
    __syncthreads();
  }
  // inverse of L by columns: X[i][c] = (delta_ic - sum_{c<=l<i} L[i][l] X[l][c]) / L[i][i]
  if (tid < kw) {
    const int c = tid;
    for (int i = c; i < kw; ++i) {
      double2 s = make_double2(i == c ? 1.0 : 0.0, 0.0);
      for (int l = c; l < i; ++l) s = csub(s, cmul(S[i][l], X[l][c]));
      X[i][c] = cscale(1.0 / S[i][i].x, s);
    }
  }
  __syncthreads();
  for (int e = tid; e < CB * CB; e += blockDim.x) {
    int i = e / CB, j = e % CB;
    if (i < kw && j < kw) {
      A[size_t(k0 + i) * m + k0 + j] = (j <= i) ? S[i][j] : make_double2(0, 0);
    }
    Dinv[e] = X[i][j];
  }
  if (tid == 0 && bad) atomicExch(info, 1);
}

// Panel below the diagonal block: L[i][k0..] = A[i][k0..] * L_kk^-H, for
// the 64-row block starting at row r0 = k0 + kw + blockIdx.x * CB.
__global__ void __launch_bounds__(256)
k_chol_panel(double2* __restrict__ A, int m, int k0, const double2* __restrict__ Dinv, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double2 P[CB][CB + 1];
  __shared__ double2 D[CB][CB + 1];
  const int kw = min(CB, m - k0);
  const int r0 = k0 + kw + blockIdx.x * CB;
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * CB; e += blockDim.x) {
    int i = e / CB, j = e % CB;
    P[i][j] = (r0 + i < m && j < kw) ? A[size_t(r0 + i) * m + k0 + j] : make_double2(0, 0);
    D[i][j] = Dinv[e];
  }
  __syncthreads();
  // out[i][j] = sum_l P[i][l] conj(D[j][l])
  for (int e = tid; e < CB * CB; e += blockDim.x) {
    int i = e / CB, j = e % CB;
    if (r0 + i >= m || j >= kw) continue;
    double2 s = make_double2(0, 0);
    for (int l = 0; l <= j; ++l) s = cadd(s, cmulc(P[i][l], D[j][l]));
    A[size_t(r0 + i) * m + k0 + j] = s;
  }
}

// Trailing update A[i][j] -= sum_l L[i][k0+l] conj(L[j][k0+l]) on the lower
// tiles of the trailing matrix (tile pair number -> (ti, tj), ti >= tj).
__global__ void __launch_bounds__(256)
k_chol_update(double2* __restrict__ A, int m, int k0, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double2 Li[CB][CB + 1];
  __shared__ double2 Lj[CB][CB + 1];
  const int kw = min(CB, m - k0);
  const int t0 = k0 + kw;
  int p = blockIdx.x, a = 0;
  while ((a + 1) * (a + 2) / 2 <= p) ++a;
  const int ti = a, tj = p - a * (a + 1) / 2;
  const int i0 = t0 + ti * CB, j0 = t0 + tj * CB;
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * CB; e += blockDim.x) {
    int r = e / CB, l = e % CB;
    Li[r][l] = (i0 + r < m && l < kw) ? A[size_t(i0 + r) * m + k0 + l] : make_double2(0, 0);
    Lj[r][l] = (j0 + r < m && l < kw) ? A[size_t(j0 + r) * m + k0 + l] : make_double2(0, 0);
  }
  __syncthreads();
  for (int e = tid; e < CB * CB; e += blockDim.x) {
    int r = e / CB, c = e % CB;
    int gi = i0 + r, gj = j0 + c;
    if (gi >= m || gj >= m || gj > gi) continue;
    double2 s = make_double2(0, 0);
    for (int l = 0; l < kw; ++l) s = cadd(s, cmulc(Li[r][l], Lj[c][l]));
    size_t idx = size_t(gi) * m + gj;
    A[idx] = csub(A[idx], s);
  }
}

// Block row ib of Linv (jb < ib), on the FP64 matrix cores:
//   Linv[ib][jb] = -Dinv[ib] * S,  S = sum_{kb=jb}^{ib-1} L[ib][kb] Linv[kb][jb]
// one workgroup per jb; Linv[ib][ib] = Dinv[ib] is written by jb == ib.
__global__ void __launch_bounds__(256)
k_tri_inv_row(const double2* __restrict__ L, double2* __restrict__ Linv, int m, int ib,
              const double2* __restrict__ Dinv_all, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using namespace mfma;
  __shared__ double2 sA[TM * KP];
  __shared__ double2 sB[TM * KP];
  __shared__ double2 Ssh[CB][CB + 1];
  const int jb = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int r0 = ib * CB;
  const double2* Di = Dinv_all + size_t(ib) * CB * CB;
  if (jb == ib) {
    for (int e = tid; e < CB * CB; e += blockDim.x) {
      int r = e / CB, c = e % CB;
      if (r0 + r < m && r0 + c < m) Linv[size_t(r0 + r) * m + r0 + c] = Di[e];
    }
    return;
  }
  Acc acc;
  zero(acc);
  for (int kb = jb; kb < ib; ++kb) {
    for (int kc = 0; kc < CB; kc += KC) {
      for (int e = tid; e < TM * KC; e += GT) {
        const int t = e / KC, k = e % KC;
        const int col = kb * CB + kc + k;            // < m since kb < ib
        sA[t * KP + k] = (r0 + t < m) ? L[size_t(r0 + t) * m + col] : make_double2(0, 0);
        sB[t * KP + k] = Linv[size_t(col) * m + jb * CB + t];
      }
      __syncthreads();
      tile<false>(acc, sA, sB, wm, wn, lane);
      __syncthreads();
    }
  }
  foreach(acc, wm, wn, lane, [&](int row, int col, double re, double im) {
    Ssh[row][col] = make_double2(re, im);
  });
  __syncthreads();
  zero(acc);
  for (int kc = 0; kc < CB; kc += KC) {
    for (int e = tid; e < TM * KC; e += GT) {
      const int t = e / KC, k = e % KC;
      sA[t * KP + k] = Di[t * CB + kc + k];
      sB[t * KP + k] = Ssh[kc + k][t];
    }
    __syncthreads();
    tile<false>(acc, sA, sB, wm, wn, lane);
    __syncthreads();
  }
  foreach(acc, wm, wn, lane, [&](int row, int col, double re, double im) {
    if (r0 + row < m && jb * CB + col < m)
      Linv[size_t(r0 + row) * m + jb * CB + col] = make_double2(-re, -im);
  });
}

__global__ void k_zero_cpx(double2* __restrict__ p, size_t n, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0, 0);
}

__global__ void k_zero(double* __restrict__ p, size_t n, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ------------------------------------------------------------------ Loewdin series
// D = A - 1 and per-block partial sums of |D_ij|^2.
__global__ void __launch_bounds__(256)
k_minus_identity(const double2* __restrict__ A, double2* __restrict__ D, int m,
                 double* __restrict__ part, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  double acc = 0.0;
  const size_t n = size_t(m) * m;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
       e += size_t(gridDim.x) * blockDim.x) {
    double2 a = A[e];
    if (e / m == e % m) a.x -= 1.0;
    D[e] = a;
    acc += a.x * a.x + a.y * a.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_sum_parts(const double* __restrict__ part, int nb, double* __restrict__ out, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  if (threadIdx.x) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  out[0] = s;
}

// P = a D + c 1
__global__ void k_axpy_identity(const double2* __restrict__ D, double a, double c,
                                double2* __restrict__ P, int m, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= size_t(m) * m) return;
  const double2 d = D[e];
  P[e] = make_double2(a * d.x + ((e / m == e % m) ? c : 0.0), a * d.y);
}

// P += c 1
__global__ void k_add_identity(double2* __restrict__ P, double c, int m, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) P[size_t(i) * m + i].x += c;
}

// ------------------------------------------------------------------ Jacobi
// Diagonalise the 64x64 pair sub-matrix of blocks (P, Q) of A (ld = mp)
// and write its unitary J (64x64, row-major, local index l < 32 -> block P).
constexpr int JT = 256;    // threads of a pair sub-problem workgroup
__global__ void __launch_bounds__(JT)
k_jacobi_pair(const double2* __restrict__ A, int mp, const int2* __restrict__ pairs,
              double2* __restrict__ Jout, int* __restrict__ rotated, double tol, int max_inner, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double2 S[JP][JP + 1];
  __shared__ double2 J[JP][JP + 1];
  __shared__ Rot rot[JB];
  __shared__ double red[JT / 64][2];
  __shared__ int done, any_rot;
  const int2 pq = pairs[blockIdx.x];
  const int tid = threadIdx.x;
  for (int e = tid; e < JP * JP; e += blockDim.x) {
    int i = e / JP, j = e % JP;
    int gi = (i < JB ? pq.x * JB + i : pq.y * JB + i - JB);
    int gj = (j < JB ? pq.x * JB + j : pq.y * JB + j - JB);
    S[i][j] = A[size_t(gi) * mp + gj];
    J[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  if (tid == 0) any_rot = 0;
  __syncthreads();
  for (int sweep = 0; sweep < max_inner; ++sweep) {
    // convergence test on the sub-matrix
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < JP * JP; e += blockDim.x) {
      int i = e / JP, j = e % JP;
      double v = S[i][j].x * S[i][j].x + S[i][j].y * S[i][j].y;
      if (i == j) dia += v; else off += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_down(off, o, 64);
      dia += __shfl_down(dia, o, 64);
    }
    if ((tid & 63) == 0) { red[tid >> 6][0] = off; red[tid >> 6][1] = dia; }
    __syncthreads();
    if (tid == 0) {
      double o = 0.0, d = 0.0;
      for (int w = 0; w < JT / 64; ++w) { o += red[w][0]; d += red[w][1]; }
      done = (o <= tol * tol * d) || (o < 1e-300);
    }
    __syncthreads();
    if (done) break;
    if (tid == 0) any_rot = 1;
    for (int r = 0; r < JP - 1; ++r) {
      if (tid < JB) {
        int p, q;
        rr_pair(JP, r, tid, p, q);
        if (p > q) { int t = p; p = q; q = t; }
        rot[tid] = make_rot(S[p][p].x, S[q][q].x, S[p][q]);
      }
      __syncthreads();
      // S <- G^H S G on 2x2 blocks (pair u rows, pair v cols)
      for (int e = tid; e < JB * JB; e += blockDim.x) {
        int u = e / JB, v = e % JB;
        int pu, qu, pv, qv;
        rr_pair(JP, r, u, pu, qu);
        rr_pair(JP, r, v, pv, qv);
        if (pu > qu) { int t = pu; pu = qu; qu = t; }
        if (pv > qv) { int t = pv; pv = qv; qv = t; }
        Rot gu = rot[u], gv = rot[v];
        double2 epu = make_double2(gu.er, gu.ei), epv = make_double2(gv.er, gv.ei);
        double2 x00 = S[pu][pv], x01 = S[pu][qv], x10 = S[qu][pv], x11 = S[qu][qv];
        // right multiply by G_v: col p' = e c col_p - s col_q ; col q' = e s col_p + c col_q
        double2 y00 = csub(cscale(gv.c, cmul(x00, epv)), cscale(gv.s, x01));
        double2 y01 = cadd(cscale(gv.s, cmul(x00, epv)), cscale(gv.c, x01));
        double2 y10 = csub(cscale(gv.c, cmul(x10, epv)), cscale(gv.s, x11));
        double2 y11 = cadd(cscale(gv.s, cmul(x10, epv)), cscale(gv.c, x11));
        // left multiply by G_u^H: row p' = conj(e) c row_p - s row_q ; row q' = conj(e) s row_p + c row_q
        S[pu][pv] = csub(cscale(gu.c, cmulc(y00, epu)), cscale(gu.s, y10));
        S[pu][qv] = csub(cscale(gu.c, cmulc(y01, epu)), cscale(gu.s, y11));
        S[qu][pv] = cadd(cscale(gu.s, cmulc(y00, epu)), cscale(gu.c, y10));
        S[qu][qv] = cadd(cscale(gu.s, cmulc(y01, epu)), cscale(gu.c, y11));
      }
      // J <- J G
      for (int e = tid; e < JP * JB; e += blockDim.x) {
        int i = e / JB, v = e % JB;
        int pv, qv;
        rr_pair(JP, r, v, pv, qv);
        if (pv > qv) { int t = pv; pv = qv; qv = t; }
        Rot gv = rot[v];
        double2 epv = make_double2(gv.er, gv.ei);
        double2 x0 = J[i][pv], x1 = J[i][qv];
        J[i][pv] = csub(cscale(gv.c, cmul(x0, epv)), cscale(gv.s, x1));
        J[i][qv] = cadd(cscale(gv.s, cmul(x0, epv)), cscale(gv.c, x1));
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (tid == 0) rotated[blockIdx.x] = any_rot;
  if (!any_rot) return;   // J = identity: the apply kernels skip this pair
  double2* out = Jout + size_t(blockIdx.x) * JP * JP;
  for (int e = tid; e < JP * JP; e += blockDim.x) out[e] = J[e / JP][e % JP];
}

// A[{Pu,Qu}][{Pv,Qv}] <- J_u^H A[..][..] J_v for the pair pairs u >= v (block
// number -> (u, v)); the mirrored block (v, u) gets the conjugate transpose,
// since A stays Hermitian.  Pairs whose J is the identity are skipped.
__global__ void __launch_bounds__(256)
k_jacobi_apply_a(double2* __restrict__ A, int mp, const int2* __restrict__ pairs,
                 const double2* __restrict__ Jall, const int* __restrict__ rotated, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double2 X[JP][JP + 1];
  __shared__ double2 M[JP][JP + 1];
  int b = blockIdx.x, u = 0;
  while ((u + 1) * (u + 2) / 2 <= b) ++u;
  const int v = b - u * (u + 1) / 2;
  const int ru = rotated[u], rv = rotated[v];
  if (!ru && !rv) return;
  const int2 pu = pairs[u], pv = pairs[v];
  const int tid = threadIdx.x;
  auto gidx = [&](int2 p, int l) { return l < JB ? p.x * JB + l : p.y * JB + l - JB; };
  const double2* Ju = Jall + size_t(u) * JP * JP;
  const double2* Jv = Jall + size_t(v) * JP * JP;
  for (int e = tid; e < JP * JP; e += blockDim.x) {
    int i = e / JP, j = e % JP;
    X[i][j] = A[size_t(gidx(pu, i)) * mp + gidx(pv, j)];
    if (rv) M[i][j] = Jv[e];
  }
  __syncthreads();
  double2 y[JE];
  if (rv) {
    for (int q = 0; q < JE; ++q) {        // Y = X Jv
      int e = tid + q * 256, i = e / JP, j = e % JP;
      double2 s = make_double2(0, 0);
      for (int l = 0; l < JP; ++l) s = cadd(s, cmul(X[i][l], M[l][j]));
      y[q] = s;
    }
  } else {
    for (int q = 0; q < JE; ++q) {
      int e = tid + q * 256;
      y[q] = X[e / JP][e % JP];
    }
  }
  __syncthreads();
  for (int q = 0; q < JE; ++q) {
    int e = tid + q * 256;
    X[e / JP][e % JP] = y[q];
    if (ru) M[e / JP][e % JP] = Ju[e];
  }
  __syncthreads();
  for (int q = 0; q < JE; ++q) {        // T = Ju^H Y
    int e = tid + q * 256, i = e / JP, j = e % JP;
    double2 s;
    if (ru) {
      s = make_double2(0, 0);
      for (int l = 0; l < JP; ++l) s = cadd(s, cconjmul(M[l][i], X[l][j]));
    } else {
      s = X[i][j];
    }
    A[size_t(gidx(pu, i)) * mp + gidx(pv, j)] = s;
    if (u != v) A[size_t(gidx(pv, j)) * mp + gidx(pu, i)] = make_double2(s.x, -s.y);
  }
}

// V[rows][{P,Q}] <- V[rows][{P,Q}] J for an RV-row block and one pair.
__global__ void __launch_bounds__(256)
k_jacobi_apply_v(double2* __restrict__ V, int mp, const int2* __restrict__ pairs,
                 const double2* __restrict__ Jall, const int* __restrict__ rotated, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double2 X[RV][JP + 1];
  __shared__ double2 M[JP][JP + 1];
  const int v = blockIdx.y, r0 = blockIdx.x * RV;
  if (!rotated[v]) return;
  const int2 pv = pairs[v];
  const int tid = threadIdx.x;
  auto gcol = [&](int l) { return l < JB ? pv.x * JB + l : pv.y * JB + l - JB; };
  const double2* Jv = Jall + size_t(v) * JP * JP;
  for (int e = tid; e < RV * JP; e += blockDim.x) {
    int i = e / JP, j = e % JP;
    X[i][j] = (r0 + i < mp) ? V[size_t(r0 + i) * mp + gcol(j)] : make_double2(0, 0);
  }
  for (int e = tid; e < JP * JP; e += blockDim.x) M[e / JP][e % JP] = Jv[e];
  __syncthreads();
  for (int e = tid; e < RV * JP; e += blockDim.x) {
    int i = e / JP, j = e % JP;
    double2 s = make_double2(0, 0);
    for (int l = 0; l < JP; ++l) s = cadd(s, cmul(X[i][l], M[l][j]));
    if (r0 + i < mp) V[size_t(r0 + i) * mp + gcol(j)] = s;
  }
}

// Off-diagonal and diagonal squared norms of A (mp x mp), per block partials.
__global__ void k_offnorm(const double2* __restrict__ A, int mp, double* __restrict__ part, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ double red[4][2];
  double off = 0.0, dia = 0.0;
  const size_t n = size_t(mp) * mp;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
       e += size_t(gridDim.x) * blockDim.x) {
    double2 a = A[e];
    double v = a.x * a.x + a.y * a.y;
    if (e / mp == e % mp) dia += v; else off += v;
  }
  for (int o = 32; o > 0; o >>= 1) {
    off += __shfl_down(off, o, 64);
    dia += __shfl_down(dia, o, 64);
  }
  if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6][0] = off; red[threadIdx.x >> 6][1] = dia; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = 0.0, d = 0.0;
    for (int w = 0; w < 4; ++w) { o += red[w][0]; d += red[w][1]; }
    part[2 * blockIdx.x] = o;
    part[2 * blockIdx.x + 1] = d;
  }
}

__global__ void k_offnorm_final(const double* __restrict__ part, int nb, double* __restrict__ out, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  if (threadIdx.x) return;
  double o = 0.0, d = 0.0;
  for (int b = 0; b < nb; ++b) { o += part[2 * b]; d += part[2 * b + 1]; }
  out[0] = o;
  out[1] = d;
}

// Pad-copy A (m x m) into Ap (mp x mp) with zero coupling, V = identity.
__global__ void k_jacobi_init(const double2* __restrict__ A, int m, double2* __restrict__ Ap,
                              double2* __restrict__ V, int mp, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= size_t(mp) * mp) return;
  int i = int(e / mp), j = int(e % mp);
  Ap[e] = (i < m && j < m) ? A[size_t(i) * m + j] : make_double2(0, 0);
  V[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
}

// Sort eigenvalues ascending (ties by index) and gather eigenvector columns.
__global__ void k_jacobi_sort(const double2* __restrict__ Ap, const double2* __restrict__ V,
                              int m, int mp, double* __restrict__ w, double2* __restrict__ Z, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int i = blockIdx.x;   // source column
  const double wi = Ap[size_t(i) * mp + i].x;
  __shared__ int rank_s;
  if (threadIdx.x == 0) rank_s = 0;
  __syncthreads();
  int cnt = 0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    double wj = Ap[size_t(j) * mp + j].x;
    if (wj < wi || (wj == wi && j < i)) ++cnt;
  }
  atomicAdd(&rank_s, cnt);
  __syncthreads();
  const int rk = rank_s;
  if (threadIdx.x == 0) w[rk] = wi;
  for (int r = threadIdx.x; r < m; r += blockDim.x) Z[size_t(r) * m + rk] = V[size_t(r) * mp + i];
}

__global__ void k_scale_columns(double2* __restrict__ X, const double* __restrict__ d, int m, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= size_t(m) * m) return;
  double s = d[e % m];
  X[e] = make_double2(s * X[e].x, s * X[e].y);
}

__global__ void k_inv_sqrt(double* __restrict__ w, int m, int* info, double floor_v, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double v = w[i];
  if (!(v > floor_v)) { atomicExch(info, 1); v = 1.0; }
  w[i] = 1.0 / sqrt(v);
}

int jacobi_dims(int m, int& nb) {
  nb = (m + JB - 1) / JB;
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  return nb * JB;
}
}  // namespace

void zero(double* p, size_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, p, n, g_launch_gate);
}

__global__ void k_identity(double2* __restrict__ A, int m, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= size_t(m) * m) return;
  A[e] = make_double2((e / m == e % m) ? 1.0 : 0.0, 0.0);
}

void identity(void* A, int m, hipStream_t st) {
  if (m <= 0) return;
  const size_t mm = size_t(m) * m;
  hipLaunchKernelGGL(k_identity, dim3(unsigned((mm + 255) / 256)), dim3(256), 0, st, (double2*)A, m, g_launch_gate);
}

__global__ void k_zero_f32(float* __restrict__ p, size_t n, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

void zero_f32(float* p, size_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero_f32, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, p, n, g_launch_gate);
}

void cholesky_inverse(void* Av, void* Linvv, int m, void* work, int* info, hipStream_t st,
                      double piv_min) {
  if (m <= 0) return;
  auto A = (double2*)Av;
  auto Linv = (double2*)Linvv;
  auto Dinv = (double2*)work;   // nblk * CB * CB
  const int nblk = (m + CB - 1) / CB;
  for (int kb = 0; kb < nblk; ++kb) {
    const int k0 = kb * CB;
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, A, m, k0,
                       Dinv + size_t(kb) * CB * CB, info, piv_min, g_launch_gate);
    const int rest = m - (k0 + min(CB, m - k0));
    if (rest > 0) {
      const int nb = (rest + CB - 1) / CB;
      hipLaunchKernelGGL(k_chol_panel, dim3(nb), dim3(256), 0, st, A, m, k0,
                         (const double2*)(Dinv + size_t(kb) * CB * CB), g_launch_gate);
      hipLaunchKernelGGL(k_chol_update, dim3(nb * (nb + 1) / 2), dim3(256), 0, st, A, m, k0, g_launch_gate);
    }
  }
  const size_t mm = size_t(m) * m;
  hipLaunchKernelGGL(k_zero_cpx, dim3(unsigned((mm + 255) / 256)), dim3(256), 0, st, Linv, mm, g_launch_gate);
  for (int ib = 0; ib < nblk; ++ib)
    hipLaunchKernelGGL(k_tri_inv_row, dim3(ib + 1), dim3(256), 0, st, (const double2*)A, Linv, m,
                       ib, (const double2*)Dinv, g_launch_gate);
}

size_t jacobi_scratch_bytes(int m) {
  int nb;
  const int mp = jacobi_dims(m, nb);
  size_t b = 0;
  b += 2 * size_t(mp) * mp * sizeof(double2);                 // Ap, V
  b += size_t(nb / 2) * JP * JP * sizeof(double2);            // J
  b += size_t(nb) * nb * sizeof(int2);                        // round-robin table
  b += size_t(nb) * sizeof(int) + 256;                        // rotated flags
  b += 4096 * sizeof(double);                                 // norm partials
  return b + 1024;
}

int jacobi_eigh(void* Av, int m, double* w, void* Zv, void* work, double tol, int max_sweeps,
                hipStream_t st) {
  if (m <= 0) return 0;
  int nb;
  const int mp = jacobi_dims(m, nb);
  const int np = nb / 2;
  char* wp = (char*)work;
  auto Ap = (double2*)wp; wp += size_t(mp) * mp * sizeof(double2);
  auto V = (double2*)wp; wp += size_t(mp) * mp * sizeof(double2);
  auto Jall = (double2*)wp; wp += size_t(np) * JP * JP * sizeof(double2);
  auto pairs = (int2*)wp; wp += size_t(nb) * nb * sizeof(int2);
  auto rotated = (int*)wp; wp += size_t(nb) * sizeof(int) + 256;
  auto norms = (double*)wp;
  // round-robin schedule of the block pairs, all rounds
  std::vector<int2> sched(size_t(nb - 1) * np);
  for (int r = 0; r < nb - 1; ++r)
    for (int i = 0; i < np; ++i) {
      const int n1 = nb - 1;
      int p = (i == 0) ? 0 : ((i + r - 1) % n1) + 1;
      int q = ((n1 - i + r - 1) % n1) + 1;
      sched[size_t(r) * np + i] = make_int2(std::min(p, q), std::max(p, q));
    }
  hipMemcpyAsync(pairs, sched.data(), sched.size() * sizeof(int2), hipMemcpyHostToDevice, st);
  const size_t mm = size_t(mp) * mp;
  hipLaunchKernelGGL(k_jacobi_init, dim3(unsigned((mm + 255) / 256)), dim3(256), 0, st,
                     (const double2*)Av, m, Ap, V, mp, g_launch_gate);
  const int nrb = 256;
  double host_norm[2];
  int sweeps = 0;
  bool done = false;
  for (; sweeps <= max_sweeps; ++sweeps) {
    hipLaunchKernelGGL(k_offnorm, dim3(nrb), dim3(256), 0, st, (const double2*)Ap, mp, norms, g_launch_gate);
    hipLaunchKernelGGL(k_offnorm_final, dim3(1), dim3(64), 0, st, (const double*)norms, nrb,
                       norms + 2 * nrb, g_launch_gate);
    hipMemcpyAsync(host_norm, norms + 2 * nrb, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    if (!std::isfinite(host_norm[0]) || !std::isfinite(host_norm[1])) return -2;
    if (host_norm[0] <= tol * tol * host_norm[1] || host_norm[0] < 1e-300) { done = true; break; }
    if (sweeps == max_sweeps) break;   // the norm after the last sweep was checked
    for (int r = 0; r < nb - 1; ++r) {
      const int2* pr = pairs + size_t(r) * np;
      hipLaunchKernelGGL(k_jacobi_pair, dim3(np), dim3(JT), 0, st, (const double2*)Ap, mp, pr,
                         Jall, rotated, tol * 1e-2, JACOBI_INNER, g_launch_gate);
      hipLaunchKernelGGL(k_jacobi_apply_a, dim3(np * (np + 1) / 2), dim3(256), 0, st, Ap, mp, pr,
                         (const double2*)Jall, (const int*)rotated, g_launch_gate);
      hipLaunchKernelGGL(k_jacobi_apply_v, dim3((mp + RV - 1) / RV, np), dim3(256), 0, st, V, mp, pr,
                         (const double2*)Jall, (const int*)rotated, g_launch_gate);
    }
  }
  hipLaunchKernelGGL(k_jacobi_sort, dim3(m), dim3(256), 0, st, (const double2*)Ap,
                     (const double2*)V, m, mp, w, (double2*)Zv, g_launch_gate);
  return done ? sweeps : -1;
}

void eig_sort(const void* D, const void* V, int m, int ld, double* w, void* Z, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_jacobi_sort, dim3(m), dim3(256), 0, st, (const double2*)D, (const double2*)V,
                     m, ld, w, (double2*)Z, g_launch_gate);
}

int loewdin_series(const void* Iv, void* Cv, void* Dv, void* Tv, int m, double max_dev,
                   double* scratch, void* part, hipStream_t st, int sq_split, double eps) {
  if (m <= 0) return 0;
  auto D = (double2*)Dv;
  const size_t mm = size_t(m) * m;
  const int nb = int(std::min<size_t>(256, (mm + 255) / 256));
  hipLaunchKernelGGL(k_minus_identity, dim3(nb), dim3(256), 0, st, (const double2*)Iv, D, m, scratch, g_launch_gate);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, (const double*)scratch, nb, scratch + nb, g_launch_gate);
  double fro2 = 0.0;
  hipMemcpyAsync(&fro2, scratch + nb, sizeof(double), hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  const double f = sqrt(fro2);
  if (!std::isfinite(f)) return -1;
  if (!(f <= max_dev)) return 0;
  // (1 + D)^-1/2 = sum_k c_k D^k, c_k = c_{k-1} (1 - 2k) / (2k); ||D||_2 <= f, so the
  // tail after p terms is below |c_{p+1}| f^{p+1} / (1 - f); stop below eps.
  double c[16];
  c[0] = 1.0;
  for (int k = 1; k < 16; ++k) c[k] = c[k - 1] * (1.0 - 2.0 * k) / (2.0 * k);
  int p = 1;
  while (p < 14 && fabs(c[p + 1]) * pow(f, p + 1) / (1.0 - f) > eps) ++p;
  // Horner: P = c_{p-1} 1 + c_p D; P <- c_k 1 + D P for k = p-2 .. 0
  auto C = (double2*)Cv, T = (double2*)Tv;
  double2* cur = (p % 2) ? C : T;   // ping-pong so that the last product lands in C
  double2* nxt = (p % 2) ? T : C;
  const unsigned ge = unsigned((mm + 255) / 256);
  hipLaunchKernelGGL(k_axpy_identity, dim3(ge), dim3(256), 0, st, (const double2*)D, c[p], c[p - 1],
                     cur, m, g_launch_gate);
  for (int k = p - 2; k >= 0; --k) {
    gemm_square(D, 0, cur, 0, nxt, m, st, part, 1, sq_split);   // a polynomial in D: Hermitian
    hipLaunchKernelGGL(k_add_identity, dim3((m + 255) / 256), dim3(256), 0, st, nxt, c[k], m, g_launch_gate);
    std::swap(cur, nxt);
  }
  return p;
}

// ------------------------------------------------------------------ device-decided steps
// The kernels below make the decisions of the host-driven steps on the
// device; they are launched without a gate and read the box's flags
// themselves.
__global__ void k_set_flag(int* __restrict__ flags, int idx, int value) {
  if (threadIdx.x == 0) flags[idx] = value;
}
__global__ void k_set_double(double* __restrict__ d, int idx, double value) {
  if (threadIdx.x == 0) d[idx] = value;
}

void set_flag(int* flags, int idx, int value, hipStream_t st) {
  hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, st, flags, idx, value);
}
void set_double(double* d, int idx, double value, hipStream_t st) {
  hipLaunchKernelGGL(k_set_double, dim3(1), dim3(64), 0, st, d, idx, value);
}

constexpr int SERIES_PMAX = 14;   // terms of the series at most (as loewdin_series)

// From ||D||_F^2 (fro2): the term count p of the series and its
// coefficients (dbl[D_SERIES + 2 ..]), the gates of the Horner steps, or the
// hand-over to the host.  Same arithmetic as loewdin_series.
__global__ void k_series_plan(const double* __restrict__ fro2, double max_dev, double eps, int pcap,
                              int* __restrict__ flags, double* __restrict__ dbl, int set) {
  if (threadIdx.x != 0) return;
  const bool active = flags[F_ACTIVE] != 0;
  const double f = sqrt(*fro2);
  int p = 0;
  if (active) {
    if (!isfinite(f) || !(f <= max_dev)) {
      flags[F_HOST] = HOST_LOEWDIN;
      flags[F_HOST_SET] = set;
      flags[F_ACTIVE] = 0;
    } else {
      double c[16];
      c[0] = 1.0;
      for (int k = 1; k < 16; ++k) c[k] = c[k - 1] * (1.0 - 2.0 * k) / (2.0 * k);
      p = 1;
      while (p < pcap && fabs(c[p + 1]) * pow(f, p + 1) / (1.0 - f) > eps) ++p;
      for (int k = 0; k < 16; ++k) dbl[D_SERIES + 2 + k] = c[k];
    }
  }
  dbl[D_SERIES] = f;
  dbl[D_SERIES + 1] = double(p);
  for (int k = 0; k <= SERIES_PMAX - 2; ++k) flags[F_SERIES + k] = (active && p > 0 && k <= p - 2) ? 1 : 0;
}

// Horner start P = c_{p-1} 1 + c_p D, written to the buffer that step p-2
// reads (buf[(p-1) % 2]); gated by the box's F_ACTIVE and run only if the
// series was planned (p > 0).
__global__ void k_series_start(const double2* __restrict__ D, const double* __restrict__ dbl,
                               double2* __restrict__ buf0, double2* __restrict__ buf1, int m,
                               const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int p = int(dbl[D_SERIES + 1]);
  if (p <= 0) return;
  const double a = dbl[D_SERIES + 2 + p], c = dbl[D_SERIES + 2 + p - 1];
  double2* P = ((p - 1) % 2) ? buf1 : buf0;
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= size_t(m) * m) return;
  const double2 d = D[e];
  P[e] = make_double2(a * d.x + ((e / m == e % m) ? c : 0.0), a * d.y);
}

// P += c_k 1 with c_k from the device.
__global__ void k_add_identity_dev(double2* __restrict__ P, const double* __restrict__ ck, int m,
                                   const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) P[size_t(i) * m + i].x += *ck;
}

void loewdin_series_dev(const void* Iv, void* Cv, void* Dv, void* Tv, int m, double max_dev,
                        double eps, double* scratch, void* part, hipStream_t st, int sq_split,
                        int* flags, double* dbl, int set) {
  if (m <= 0) return;
  auto D = (double2*)Dv;
  const size_t mm = size_t(m) * m;
  const int nb = int(std::min<size_t>(256, (mm + 255) / 256));
  const int* active = flags + F_ACTIVE;
  {
    GateScope g(active);
    hipLaunchKernelGGL(k_minus_identity, dim3(nb), dim3(256), 0, st, (const double2*)Iv, D, m, scratch, g_launch_gate);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, (const double*)scratch, nb, scratch + nb, g_launch_gate);
  }
  // the most terms any accepted norm (f <= max_dev) can need, plus one:
  // Horner steps beyond those are never taken and are not captured
  double c[16];
  c[0] = 1.0;
  for (int k = 1; k < 16; ++k) c[k] = c[k - 1] * (1.0 - 2.0 * k) / (2.0 * k);
  int pmax = 1;
  while (pmax < SERIES_PMAX && fabs(c[pmax + 1]) * pow(max_dev, pmax + 1) / (1.0 - max_dev) > eps)
    ++pmax;
  const int pcap = std::min(pmax + 1, SERIES_PMAX);
  hipLaunchKernelGGL(k_series_plan, dim3(1), dim3(64), 0, st, (const double*)(scratch + nb), max_dev,
                     eps, pcap, flags, dbl, set);
  // buf[0] = C receives the last Horner step (k = 0), buf[1] = T
  auto C = (double2*)Cv, T = (double2*)Tv;
  double2* buf[2] = {C, T};
  const unsigned ge = unsigned((mm + 255) / 256);
  hipLaunchKernelGGL(k_series_start, dim3(ge), dim3(256), 0, st, (const double2*)D,
                     (const double*)dbl, C, T, m, active);
  for (int k = pcap - 2; k >= 0; --k) {
    GateScope g(flags + F_SERIES + k);
    gemm_square(D, 0, buf[(k + 1) % 2], 0, buf[k % 2], m, st, part, 1, sq_split);
    hipLaunchKernelGGL(k_add_identity_dev, dim3((m + 255) / 256), dim3(256), 0, st, buf[k % 2],
                       (const double*)(dbl + D_SERIES + 2 + k), m, g_launch_gate);
  }
}

// One workgroup of 256 threads: Delta-eps from the residual norms of the
// occupied states of every set, in a fixed order.
struct R2Sets {
  const double* r2[64];
  int nocc[64];
};
__global__ void __launch_bounds__(256)
k_iteration_end(R2Sets sets, int nset, int count, int* __restrict__ flags, double* __restrict__ dbl) {
  if (flags[F_ACTIVE] == 0) return;
  __shared__ double buf[256];
  double acc = 0.0;
  for (int s = 0; s < nset; ++s)
    for (int a = threadIdx.x; a < sets.nocc[s]; a += 256) acc += sets.r2[s][a];
  buf[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) buf[threadIdx.x] += buf[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double de = sqrt(buf[0] / double(count > 0 ? count : 1));
    dbl[D_DE] = de;
    flags[F_ITER] += 1;
    if (!isfinite(de)) {
      flags[F_HOST] = HOST_NAN;
      flags[F_HOST_SET] = 0;
      flags[F_ACTIVE] = 0;
    } else if (dbl[D_TOL] > 0.0 && de <= dbl[D_TOL]) {
      flags[F_CONV] = 1;
      flags[F_ACTIVE] = 0;
    }
  }
}

void iteration_end(const double* const* r2, const int* nocc, int nset, int count, int* flags,
                   double* dbl, hipStream_t st) {
  R2Sets sets{};
  const int ns = std::min(nset, 64);
  for (int s = 0; s < ns; ++s) {
    sets.r2[s] = r2[s];
    sets.nocc[s] = nocc[s];
  }
  hipLaunchKernelGGL(k_iteration_end, dim3(1), dim3(256), 0, st, sets, ns, count, flags, dbl);
}

// Gauge of the paper-literal update.  info[3 c .. 3 c + 2] = (start a, size k,
// offset o) of the cluster holding column c; a cluster's k x k diagonal
// block lives at packed[o ..] row-major.
__global__ void k_gauge_gather(const double2* __restrict__ Z, int m, const int* __restrict__ info,
                               double2* __restrict__ packed, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int c = blockIdx.y;
  const int a = info[3 * c], k = info[3 * c + 1], o = info[3 * c + 2];
  for (int r = threadIdx.x; r < k; r += blockDim.x)
    packed[size_t(o) + size_t(r) * k + (c - a)] = Z[size_t(a + r) * m + c];
}

// out[:, c] = sum_l Z[:, a + l] Q[l][c - a] over the cluster of column c.
__global__ void k_gauge_apply(const double2* __restrict__ Z, int m, const int* __restrict__ info,
                              const double2* __restrict__ Q, double2* __restrict__ out, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int c = blockIdx.y;
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= m) return;
  const int a = info[3 * c], k = info[3 * c + 1], o = info[3 * c + 2];
  double2 acc = make_double2(0.0, 0.0);
  for (int l = 0; l < k; ++l) acc = cadd(acc, cmul(Z[size_t(row) * m + a + l], Q[size_t(o) + size_t(l) * k + (c - a)]));
  out[size_t(row) * m + c] = acc;
}

void gauge_gather(const void* Z, int m, const int* info, void* packed, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_gauge_gather, dim3(1, m), dim3(64), 0, st, (const double2*)Z, m, info,
                     (double2*)packed, g_launch_gate);
}

void gauge_apply(const void* Z, int m, const int* info, const void* Q, void* out, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_gauge_apply, dim3((m + 255) / 256, m), dim3(256), 0, st, (const double2*)Z, m,
                     info, (const double2*)Q, (double2*)out, g_launch_gate);
}

void scale_columns(void* X, const double* d, int m, hipStream_t st) {
  const size_t mm = size_t(m) * m;
  hipLaunchKernelGGL(k_scale_columns, dim3(unsigned((mm + 255) / 256)), dim3(256), 0, st,
                     (double2*)X, d, m, g_launch_gate);
}

void inv_sqrt(double* w, int m, int* info, hipStream_t st, double floor_v) {
  hipLaunchKernelGGL(k_inv_sqrt, dim3((m + 255) / 256), dim3(256), 0, st, w, m, info, floor_v, g_launch_gate);
}

}  // namespace sky
