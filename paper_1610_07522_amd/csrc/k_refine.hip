// Hermitian eigensolver of the subspace Hamiltonian by eigenvector
// refinement (Sec. 3.3.2, step 3b: H' = Z Lambda Z^H).
//
// After the first iterations of the damped-gradient method the orthonormalised
// subspace Hamiltonian H' is close to diagonal: the previous states were its
// Ritz vectors, and one damped step couples them only weakly.  Its spectrum
// is full of (near-)degenerate multiplets, but the multiplets are small.  The
// solver refines X (start X = 1) towards X^H X = 1, X^H H' X = diagonal with a
// Newton-type update on FP64 matrix cores:
//
//   R = 1 - X^H X,  S = X^H H' X (both symmetrised),
//   lam_i = Re S_ii / (1 - Re R_ii);
//   sort by lam; cut the sorted order into contiguous clusters so that every
//   pair (i, j) in different clusters is weakly coupled,
//   |S_ij + lam R_ij| <= THETA |lam_j - lam_i| (both orientations);
//   diagonalise each cluster block of (1 + R/2) S (1 + R/2) exactly (cyclic
//   Jacobi in one workgroup, unitary W_c; B = blockdiag(W_c) in sorted order);
//   in the rotated basis (S2 = B^H S B, R2 = B^H R B, lam2 from its diagonal)
//   E_ab = (S2_ab + lam2_b R2_ab) / (lam2_b - lam2_a) across clusters,
//   E_ab = R2_ab / 2 inside a cluster and for couplings at the rounding floor;
//   X <- X P B (1 + E + E^2 / 2)   (P: sorted -> original order).
//
// The cross-cluster part of E is the first-order eigenvector correction and
// the in-cluster part the first-order orthonormality correction; the E^2/2
// term makes the update unitary to second order, so that the off-diagonal
// norm and the orthonormality defect fall quadratically.  Convergence: the
// relative off-diagonal Frobenius norm of S below tol and max |R_ij| below
// orth.  A cluster wider than KMAX, a non-finite value or no convergence
// within the iteration limit returns a failure, and the caller falls back to
// the blocked Jacobi solver.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "jacobi_rot.h"
#include "sky_kernels.h"

namespace sky {

namespace {
using namespace jrot;

constexpr int KMAX = 48;            // widest cluster diagonalised in one workgroup (LDS: 3 x 48 x 49 x 16 B)
constexpr double THETA = 0.03;      // weak-coupling ratio |coupling| / |gap|
constexpr double E_CLAMP = 0.25;    // bound on one update coefficient
constexpr int CHECK_BLOCKS = 256;

// lam[i] = Re S_ii / (1 - Re R_ii)  (R may be null: R = 0); clears *emax.
__global__ void k_ref_lambda(const double2* __restrict__ S, const double2* __restrict__ R, int m,
                             double* __restrict__ lam, unsigned long long* __restrict__ emax, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *emax = 0ull;
  if (i >= m) return;
  const double r = R ? R[size_t(i) * m + i].x : 0.0;
  lam[i] = S[size_t(i) * m + i].x / (1.0 - r);
}

// rank[i] = position of i in ascending (lam, index) order; order[rank] = i.
// A workgroup ranks 64 values; each of its RANK_SPLIT waves counts over one
// slice of the others, and the slice counts are summed in LDS.
constexpr int RANK_SPLIT = 16;
__global__ void __launch_bounds__(64 * RANK_SPLIT)
k_ref_rank(const double* __restrict__ lam, int m, int* __restrict__ rank,
           int* __restrict__ order, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ int cnt[RANK_SPLIT][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const double li = i < m ? lam[i] : 0.0;
  const int per = (m + RANK_SPLIT - 1) / RANK_SPLIT;
  const int j0 = min(m, wv * per), j1 = min(m, j0 + per);
  int r = 0;
  if (i < m)
    for (int j = j0; j < j1; ++j) {
      const double lj = lam[j];
      r += (lj < li || (lj == li && j < i)) ? 1 : 0;
    }
  cnt[wv][lane] = r;
  __syncthreads();
  if (wv != 0 || i >= m) return;
  int t = 0;
  for (int k = 0; k < RANK_SPLIT; ++k) t += cnt[k][lane];
  rank[i] = t;
  order[t] = i;
}

// reach[rank[i]] = largest sorted position strongly coupled to i (or its own).
__global__ void __launch_bounds__(256)
k_ref_reach(const double2* __restrict__ S, const double2* __restrict__ R, const double* __restrict__ lam,
            const int* __restrict__ rank, int m, double theta, const double* __restrict__ taup,
            int* __restrict__ reach, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int i = blockIdx.x;
  const double tau = *taup;
  const double li = lam[i];
  const int ri = rank[i];
  int best = ri;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const int rj = rank[j];
    if (rj <= best) continue;
    const double lj = lam[j];
    const double2 s = S[size_t(i) * m + j];
    const double2 r = R ? R[size_t(i) * m + j] : make_double2(0.0, 0.0);
    const double g1 = hypot(s.x + lj * r.x, s.y + lj * r.y);
    const double g2 = hypot(s.x + li * r.x, s.y + li * r.y);
    // couplings at the noise floor tau of H' never join a cluster
    if (fmax(g1, g2) > tau && fmax(g1, g2) > theta * fabs(lj - li)) best = rj;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o));
  __shared__ int wb[4];
  if ((threadIdx.x & 63) == 0) wb[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) reach[ri] = max(max(wb[0], wb[1]), max(wb[2], wb[3]));
}

// Contiguous clusters of sorted positions: a cut after position a when no
// strong coupling crosses it (prefix max of reach == a).  Per position:
// cstart (first position of its cluster), csize, cslot (index into the
// cluster list, -1 for singletons).  The list holds (start, size) of every
// cluster of two to KMAX positions; info[0] = list length, info[1] = widest
// cluster found.
// One workgroup of 1024 threads, chunked scans; pm (m ints) holds the
// prefix maximum.
__global__ void __launch_bounds__(1024)
k_ref_clusters(const int* __restrict__ reach, int m, int* __restrict__ pm, int* __restrict__ cstart,
               int* __restrict__ csize, int* __restrict__ cslot, int2* __restrict__ clist,
               int* __restrict__ info, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ int tmax[1024], tcut[1024];
  __shared__ int ncl, widest;
  const int t = threadIdx.x, T = blockDim.x;
  const int chunk = (m + T - 1) / T;
  const int a0 = min(m, t * chunk), a1 = min(m, a0 + chunk);
  if (t == 0) { ncl = 0; widest = 1; }
  // pass 1: chunk prefix max of reach
  int mx = -1;
  for (int a = a0; a < a1; ++a) mx = max(mx, reach[a]);
  tmax[t] = mx;
  __syncthreads();
  if (t == 0)
    for (int u = 1; u < T; ++u) tmax[u] = max(tmax[u], tmax[u - 1]);
  __syncthreads();
  // pass 2: cuts; last cut before each chunk
  int run = t ? tmax[t - 1] : -1;
  int lastcut = -1;
  for (int a = a0; a < a1; ++a) {
    run = max(run, reach[a]);
    if (run == a) lastcut = a;
    pm[a] = run;
  }
  tcut[t] = lastcut;
  __syncthreads();
  if (t == 0)
    for (int u = 1; u < T; ++u) tcut[u] = max(tcut[u], tcut[u - 1]);
  __syncthreads();
  // pass 3: start of each position's cluster = last cut before it + 1
  int prevcut = t ? tcut[t - 1] : -1;
  for (int a = a0; a < a1; ++a) {
    const bool cut = pm[a] == a;
    const int st = prevcut + 1;
    if (cut) {
      const int k = a - st + 1;
      atomicMax(&widest, k);
      if (k > 1 && k <= KMAX) {
        const int slot = atomicAdd(&ncl, 1);
        clist[slot] = make_int2(st, k);
        for (int b = st; b <= a; ++b) {
          cstart[b] = st;
          csize[b] = k;
          cslot[b] = slot;
        }
      } else {
        // singletons; a cluster wider than KMAX is only reported (info[1]),
        // its members stay singletons so every later access stays in bounds
        for (int b = st; b <= a; ++b) {
          cstart[b] = b;
          csize[b] = 1;
          cslot[b] = -1;
        }
      }
      prevcut = a;
    }
  }
  __syncthreads();
  if (t == 0) { info[0] = ncl; info[1] = widest; }
}

// W[c] (KMAX x KMAX, leading k x k block used) diagonalises the Hermitian
// part of S on cluster c (rows and columns order[start .. start+k)), taken in
// the first-order orthonormalised basis (1 + R/2): for an exactly degenerate
// multiplet the metric defect lam R would otherwise decide the rotation.
// Together with the in-cluster update term R/2 the transform of the cluster
// is (1 + R/2) W.  Cyclic Jacobi in LDS, round-robin ordering, the same
// rotations as the blocked solver's pair sub-problems.
__global__ void __launch_bounds__(256)
k_ref_cluster_eig(const double2* __restrict__ S, const double2* __restrict__ R, int m,
                  const int* __restrict__ order, const int2* __restrict__ clist,
                  const int* __restrict__ info, double2* __restrict__ W, double tol, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int c = blockIdx.x;
  if (c >= info[0]) return;
  const int2 cs = clist[c];
  const int k = cs.y;
  if (k > KMAX) return;   // reported through info[1]; the caller falls back
  const int np = (k + 1) & ~1, nh = np / 2;
  __shared__ double2 M[KMAX][KMAX + 1];
  __shared__ double2 J[KMAX][KMAX + 1];
  __shared__ double2 P[KMAX][KMAX + 1];
  __shared__ Rot rot[KMAX / 2];
  __shared__ int idx[KMAX];
  __shared__ double red[4][2];
  __shared__ int done;
  const int tid = threadIdx.x;
  if (tid < k) idx[tid] = order[cs.x + tid];
  __syncthreads();
  for (int e = tid; e < np * np; e += blockDim.x) {
    const int i = e / np, j = e % np;
    double2 v = make_double2(0.0, 0.0), rv = make_double2(0.0, 0.0);
    if (i < k && j < k) {
      const double2 a = S[size_t(idx[i]) * m + idx[j]], b = S[size_t(idx[j]) * m + idx[i]];
      v = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      if (R) {
        const double2 c = R[size_t(idx[i]) * m + idx[j]], d = R[size_t(idx[j]) * m + idx[i]];
        rv = make_double2(0.5 * (c.x + d.x), 0.5 * (c.y - d.y));
      }
    }
    M[i][j] = v;
    J[i][j] = rv;
  }
  __syncthreads();
  if (R) {
    // first-order Loewdin: M <- (1 + R/2) M (1 + R/2), the cluster block in
    // the orthonormalised basis (R is the metric defect 1 - X^H X there)
    for (int e = tid; e < np * np; e += blockDim.x) {
      const int i = e / np, j = e % np;
      double2 acc = M[i][j];
      for (int l = 0; l < np; ++l) acc = cadd(acc, cscale(0.5, cmul(M[i][l], J[l][j])));
      P[i][j] = acc;
    }
    __syncthreads();
    for (int e = tid; e < np * np; e += blockDim.x) {
      const int i = e / np, j = e % np;
      double2 acc = P[i][j];
      for (int l = 0; l < np; ++l) acc = cadd(acc, cscale(0.5, cmul(J[i][l], P[l][j])));
      M[i][j] = acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < np * np; e += blockDim.x) {
    const int i = e / np, j = e % np;
    J[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int sweep = 0; sweep < 16; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < np * np; e += blockDim.x) {
      const int i = e / np, j = e % np;
      const double v = M[i][j].x * M[i][j].x + M[i][j].y * M[i][j].y;
      if (i == j) dia += v; else off += v;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_down(off, o, 64);
      dia += __shfl_down(dia, o, 64);
    }
    if ((tid & 63) == 0) { red[tid >> 6][0] = off; red[tid >> 6][1] = dia; }
    __syncthreads();
    if (tid == 0) {
      const double o = red[0][0] + red[1][0] + red[2][0] + red[3][0];
      const double d = red[0][1] + red[1][1] + red[2][1] + red[3][1];
      done = (o <= tol * tol * d) || (o < 1e-300);
    }
    __syncthreads();
    if (done) break;
    for (int r = 0; r < np - 1; ++r) {
      if (tid < nh) {
        int p, q;
        rr_pair(np, r, tid, p, q);
        if (p > q) { const int t = p; p = q; q = t; }
        rot[tid] = make_rot(M[p][p].x, M[q][q].x, M[p][q]);
      }
      __syncthreads();
      // M <- G^H M G on the 2x2 blocks (rotation u rows, rotation v columns)
      for (int e = tid; e < nh * nh; e += blockDim.x) {
        const int u = e / nh, v = e % nh;
        int pu, qu, pv, qv;
        rr_pair(np, r, u, pu, qu);
        rr_pair(np, r, v, pv, qv);
        if (pu > qu) { const int t = pu; pu = qu; qu = t; }
        if (pv > qv) { const int t = pv; pv = qv; qv = t; }
        const Rot gu = rot[u], gv = rot[v];
        const double2 epu = make_double2(gu.er, gu.ei), epv = make_double2(gv.er, gv.ei);
        const double2 x00 = M[pu][pv], x01 = M[pu][qv], x10 = M[qu][pv], x11 = M[qu][qv];
        const double2 y00 = csub(cscale(gv.c, cmul(x00, epv)), cscale(gv.s, x01));
        const double2 y01 = cadd(cscale(gv.s, cmul(x00, epv)), cscale(gv.c, x01));
        const double2 y10 = csub(cscale(gv.c, cmul(x10, epv)), cscale(gv.s, x11));
        const double2 y11 = cadd(cscale(gv.s, cmul(x10, epv)), cscale(gv.c, x11));
        M[pu][pv] = csub(cscale(gu.c, cmulc(y00, epu)), cscale(gu.s, y10));
        M[pu][qv] = csub(cscale(gu.c, cmulc(y01, epu)), cscale(gu.s, y11));
        M[qu][pv] = cadd(cscale(gu.s, cmulc(y00, epu)), cscale(gu.c, y10));
        M[qu][qv] = cadd(cscale(gu.s, cmulc(y01, epu)), cscale(gu.c, y11));
      }
      // J <- J G
      for (int e = tid; e < np * nh; e += blockDim.x) {
        const int i = e / nh, v = e % nh;
        int pv, qv;
        rr_pair(np, r, v, pv, qv);
        if (pv > qv) { const int t = pv; pv = qv; qv = t; }
        const Rot gv = rot[v];
        const double2 epv = make_double2(gv.er, gv.ei);
        const double2 x0 = J[i][pv], x1 = J[i][qv];
        J[i][pv] = csub(cscale(gv.c, cmul(x0, epv)), cscale(gv.s, x1));
        J[i][qv] = cadd(cscale(gv.s, cmul(x0, epv)), cscale(gv.c, x1));
      }
      __syncthreads();
    }
  }
  double2* out = W + size_t(c) * KMAX * KMAX;
  for (int e = tid; e < k * k; e += blockDim.x) out[(e / k) * KMAX + e % k] = J[e / k][e % k];
}

// sum_{s<ka, u<kb} conj(Wa[s][ta]) M[order[sa+s]][order[sb+u]] Wb[u][tb]
// (a null W is the 1x1 identity of a singleton).
__device__ inline double2 sandwich(const double2* __restrict__ M, int m, const int* __restrict__ order,
                                   const double2* Wa, int sa, int ka, int ta,
                                   const double2* Wb, int sb, int kb, int tb) {
  double2 tot = make_double2(0.0, 0.0);
  for (int s = 0; s < ka; ++s) {
    const double2* row = M + size_t(order[sa + s]) * m;
    double2 acc = make_double2(0.0, 0.0);
    for (int u = 0; u < kb; ++u) {
      const double2 x = row[order[sb + u]];
      acc = cadd(acc, Wb ? cmul(x, Wb[u * KMAX + tb]) : x);
    }
    tot = cadd(tot, Wa ? cconjmul(Wa[s * KMAX + ta], acc) : acc);
  }
  return tot;
}

struct Clusters {
  const int *order, *cstart, *csize, *cslot;
  const double2* W;
  __device__ const double2* w(int a) const {
    return cslot[a] >= 0 ? W + size_t(cslot[a]) * KMAX * KMAX : nullptr;
  }
};

// lam2[a] = Re S2_aa / (1 - Re R2_aa) in the cluster-rotated sorted basis.
__global__ void k_ref_lambda2(const double2* __restrict__ S, const double2* __restrict__ R, int m,
                              Clusters cl, double* __restrict__ lam2, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= m) return;
  const int s0 = cl.cstart[a], k = cl.csize[a];
  const double2* Wa = cl.w(a);
  const double s2 = sandwich(S, m, cl.order, Wa, s0, k, a - s0, Wa, s0, k, a - s0).x;
  const double r2 = R ? sandwich(R, m, cl.order, Wa, s0, k, a - s0, Wa, s0, k, a - s0).x : 0.0;
  lam2[a] = s2 / (1.0 - r2);
}

// E in the cluster-rotated sorted basis (m x m, row a, column b), and
// *emax = max |E_ab|.  A pair of
// different clusters whose coupling (both orientations) is at the rounding
// floor tau of the products is converged: it gets the orthonormality term
// only.  (Its first-order coefficient would be rounding noise over a gap
// that can itself be at rounding level, e.g. an exact Kramers pair, and would
// rotate the pair at random by up to THETA on every step.)
__global__ void __launch_bounds__(256)
k_ref_update(const double2* __restrict__ S, const double2* __restrict__ R, int m, Clusters cl,
             const double* __restrict__ lam2, const double* __restrict__ taup,
             double2* __restrict__ E, unsigned long long* __restrict__ emax, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const double tau = *taup;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  double mag = 0.0;
  if (b < m) {
    const int sa = cl.cstart[a], ka = cl.csize[a], sb = cl.cstart[b], kb = cl.csize[b];
    const double2 *Wa = cl.w(a), *Wb = cl.w(b);
    double2 e = make_double2(0.0, 0.0);
    if (sa == sb) {
      if (R) e = cscale(0.5, sandwich(R, m, cl.order, Wa, sa, ka, a - sa, Wb, sb, kb, b - sb));
    } else {
      const double2 s2 = sandwich(S, m, cl.order, Wa, sa, ka, a - sa, Wb, sb, kb, b - sb);
      const double2 r2 = R ? sandwich(R, m, cl.order, Wa, sa, ka, a - sa, Wb, sb, kb, b - sb)
                           : make_double2(0.0, 0.0);
      const double2 gb = cadd(s2, cscale(lam2[b], r2)), ga = cadd(s2, cscale(lam2[a], r2));
      const double den = lam2[b] - lam2[a];
      if (fmax(hypot(gb.x, gb.y), hypot(ga.x, ga.y)) <= tau) {
        e = cscale(0.5, r2);   // coupling at the noise floor: orthonormality only
      } else if (den != 0.0) {
        e = cscale(1.0 / den, gb);
        const double em = hypot(e.x, e.y);
        if (em > E_CLAMP) e = cscale(E_CLAMP / em, e);
      }
    }
    E[size_t(a) * m + b] = e;
    mag = hypot(e.x, e.y);
  }
  // largest |E_ab| (bit patterns of non-negative doubles order like integers)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mag = fmax(mag, __shfl_xor(mag, o));
  if ((threadIdx.x & 63) == 0) atomicMax(emax, (unsigned long long)__double_as_longlong(mag));
}

// k_ref_update with one workgroup per sorted row a: the row a of B^H S (and
// B^H R), in the original column order, is formed once in LDS from the ka
// rows of a's cluster (coalesced reads), and column b then combines the kb
// entries of its own cluster from LDS.  Same E and *emax; the two sums of the
// sandwich are taken in the other order.  Dynamic LDS: (R ? 2 : 1) * m
// complex values.
template <bool HAS_R>
__global__ void __launch_bounds__(256)
k_ref_update_rows(const double2* __restrict__ S, const double2* __restrict__ R, int m, Clusters cl,
                  const double* __restrict__ lam2, const double* __restrict__ taup,
                  double2* __restrict__ E, unsigned long long* __restrict__ emax,
                  const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  extern __shared__ double2 ref_row[];
  double2* srow = ref_row;
  double2* rrow = ref_row + m;
  const double tau = *taup;
  const int a = blockIdx.x;
  const int sa = cl.cstart[a], ka = cl.csize[a], ta = a - sa;
  const double2* Wa = cl.w(a);
  for (int col = threadIdx.x; col < m; col += blockDim.x) {
    double2 sv = make_double2(0.0, 0.0), rv = make_double2(0.0, 0.0);
    for (int t = 0; t < ka; ++t) {
      const size_t o = size_t(cl.order[sa + t]) * m + col;
      if (Wa) {
        const double2 w = Wa[t * KMAX + ta];
        sv = cadd(sv, cconjmul(w, S[o]));
        if (HAS_R) rv = cadd(rv, cconjmul(w, R[o]));
      } else {
        sv = S[o];
        if (HAS_R) rv = R[o];
      }
    }
    srow[col] = sv;
    if (HAS_R) rrow[col] = rv;
  }
  __syncthreads();
  const double la = lam2[a];
  double mag = 0.0;
  for (int b = threadIdx.x; b < m; b += blockDim.x) {
    const int sb = cl.cstart[b], kb = cl.csize[b], tb = b - sb;
    const double2* Wb = cl.w(b);
    double2 s2 = make_double2(0.0, 0.0), r2 = make_double2(0.0, 0.0);
    for (int u = 0; u < kb; ++u) {
      const int c = cl.order[sb + u];
      if (Wb) {
        const double2 w = Wb[u * KMAX + tb];
        s2 = cadd(s2, cmul(srow[c], w));
        if (HAS_R) r2 = cadd(r2, cmul(rrow[c], w));
      } else {
        s2 = srow[c];
        if (HAS_R) r2 = rrow[c];
      }
    }
    double2 e = make_double2(0.0, 0.0);
    if (sa == sb) {
      if (HAS_R) e = cscale(0.5, r2);
    } else {
      const double lb = lam2[b];
      const double2 gb = cadd(s2, cscale(lb, r2)), ga = cadd(s2, cscale(la, r2));
      const double den = lb - la;
      if (fmax(hypot(gb.x, gb.y), hypot(ga.x, ga.y)) <= tau) {
        e = cscale(0.5, r2);   // coupling at the noise floor: orthonormality only
      } else if (den != 0.0) {
        e = cscale(1.0 / den, gb);
        const double em = hypot(e.x, e.y);
        if (em > E_CLAMP) e = cscale(E_CLAMP / em, e);
      }
    }
    E[size_t(a) * m + b] = e;
    mag = fmax(mag, hypot(e.x, e.y));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mag = fmax(mag, __shfl_xor(mag, o));
  if ((threadIdx.x & 63) == 0) atomicMax(emax, (unsigned long long)__double_as_longlong(mag));
}

constexpr size_t REF_ROW_LDS_MAX = 65536;   // dynamic LDS of k_ref_update_rows at most

// E and *emax of one refinement step: by rows through LDS where two rows of
// m complex values fit, else one thread per entry.
void ref_update(const double2* Sp, const double2* Rp, int m, const Clusters& cl, const double* lam2,
                const double* tau, double2* E, unsigned long long* emax, hipStream_t st) {
  const size_t lds = size_t(Rp ? 2 : 1) * m * sizeof(double2);
  if (lds <= REF_ROW_LDS_MAX) {
    if (Rp)
      hipLaunchKernelGGL(k_ref_update_rows<true>, dim3(unsigned(m)), dim3(256), lds, st, Sp, Rp, m, cl,
                         lam2, tau, E, emax, g_launch_gate);
    else
      hipLaunchKernelGGL(k_ref_update_rows<false>, dim3(unsigned(m)), dim3(256), lds, st, Sp, Rp, m, cl,
                         lam2, tau, E, emax, g_launch_gate);
  } else {
    const unsigned gm = unsigned((m + 255) / 256);
    hipLaunchKernelGGL(k_ref_update, dim3(gm, unsigned(m)), dim3(256), 0, st, Sp, Rp, m, cl, lam2, tau,
                       E, emax, g_launch_gate);
  }
}

// Q[order[s]][b] = sum_{t in cluster(s)} W[s - c][t - c] (delta_tb + E_tb + E2_tb / 2)
// (E2 null, or e2flag pointing at 0: the second-order term is below rounding
// and left out).
__global__ void __launch_bounds__(256)
k_ref_build_q(const double2* __restrict__ E, const double2* __restrict__ E2v, const int* __restrict__ e2flag,
              int m, Clusters cl, double2* __restrict__ Q, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const double2* E2 = (e2flag == nullptr || *e2flag != 0) ? E2v : nullptr;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (b >= m) return;
  const int c = cl.cstart[s], k = cl.csize[s];
  const double2* Wc = cl.w(s);
  double2 acc = make_double2(0.0, 0.0);
  for (int t = 0; t < k; ++t) {
    const size_t at = size_t(c + t) * m + b;
    double2 q = E2 ? cadd(E[at], cscale(0.5, E2[at])) : E[at];
    if (c + t == b) q.x += 1.0;
    acc = cadd(acc, Wc ? cmul(Wc[(s - c) * KMAX + t], q) : q);
  }
  Q[size_t(cl.order[s]) * m + b] = acc;
}

// Whether the step forms E^2/2: max |E| above e2skip (below, the term is
// under the precision the refinement works to).  Decided on the device (the
// flag gates the E^2 product and tells k_ref_build_q to use it); 0 when the
// run flag is off.
__global__ void k_ref_e2_flag(const unsigned long long* __restrict__ emax, const int* __restrict__ run,
                              double e2skip, int* __restrict__ flag) {
  if (threadIdx.x != 0) return;
  const double em = __longlong_as_double((long long)*emax);
  *flag = ((run == nullptr || *run != 0) && !(em <= e2skip)) ? 1 : 0;
}

// S <- (S + S^H) / 2 and R <- 1 - (G + G^H) / 2 in place (R holds G = X^H X
// on entry), with per-block partial norms: off-diagonal and diagonal
// Frobenius squares of S, max |R_ij|.  The products are Hermitian only up to
// rounding, and the update divides the anti-Hermitian part by eigenvalue
// gaps: without the symmetrisation it stalls the orthonormality near 1e-11.
__global__ void __launch_bounds__(256)
k_ref_check(double2* __restrict__ S, double2* __restrict__ R, int m,
            const double* __restrict__ taup, double* __restrict__ part, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const double tau = *taup;
  double off = 0.0, dia = 0.0, rmax = 0.0;
  const size_t n = size_t(m) * m;
  for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
       e += size_t(gridDim.x) * blockDim.x) {
    const int i = int(e / m), j = int(e % m);
    if (i < j) continue;
    double rg;
    if (i == j) {
      const double sd = S[e].x;
      S[e] = make_double2(sd, 0.0);
      dia += sd * sd;
      const double r = 1.0 - R[e].x;
      R[e] = make_double2(r, 0.0);
      rg = fabs(r);
    } else {
      const size_t et = size_t(j) * m + i;
      const double2 a = S[e], b = S[et];
      const double2 sv = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
      S[e] = sv;
      S[et] = make_double2(sv.x, -sv.y);
      // couplings at the noise floor of H' count as converged (not rotated)
      const double s2 = sv.x * sv.x + sv.y * sv.y;
      if (s2 > tau * tau) off += 2.0 * s2;
      const double2 ga = R[e], gb = R[et];
      const double2 r = make_double2(-0.5 * (ga.x + gb.x), -0.5 * (ga.y - gb.y));
      R[e] = r;
      R[et] = make_double2(r.x, -r.y);
      rg = hypot(r.x, r.y);
    }
    rmax = (rg > rmax || rg != rg) ? rg : rmax;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    off += __shfl_down(off, o, 64);
    dia += __shfl_down(dia, o, 64);
    const double t = __shfl_down(rmax, o, 64);
    rmax = (t > rmax || t != t) ? t : rmax;
  }
  __shared__ double red[4][3];
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = off;
    red[threadIdx.x >> 6][1] = dia;
    red[threadIdx.x >> 6][2] = rmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = 0.0, d = 0.0, r = 0.0;
    for (int w = 0; w < 4; ++w) {
      o += red[w][0];
      d += red[w][1];
      r = (red[w][2] > r || red[w][2] != red[w][2]) ? red[w][2] : r;
    }
    part[3 * blockIdx.x] = o;
    part[3 * blockIdx.x + 1] = d;
    part[3 * blockIdx.x + 2] = r;
  }
}

// tau = noise * rms of Re A_ii (one workgroup of 256 threads).
__global__ void __launch_bounds__(256)
k_ref_diag2(const double2* __restrict__ A, int m, double noise, double* __restrict__ tau, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  double v = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double d = A[size_t(i) * m + i].x;
    v += d * d;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) tau[0] = noise * sqrt((red[0] + red[1] + red[2] + red[3]) / m);
}

// tau = noise * rms eigenvalue from the diagonal norm of the last check.
__global__ void k_ref_tau(const double* __restrict__ norms, int m, double noise,
                          double* __restrict__ tau, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  if (threadIdx.x == 0) tau[0] = noise * sqrt(norms[1] / m);
}

// Sums of the check's block partials over 64 lanes (lane t takes blocks
// t, t + 64, ... in order, then a fixed butterfly), NaN-propagating max.
__global__ void k_ref_check_final(const double* __restrict__ part, int nb, double* __restrict__ out, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int t = threadIdx.x;
  if (t >= 64) return;
  double o = 0.0, d = 0.0, r = 0.0;
  for (int b = t; b < nb; b += 64) {
    o += part[3 * b];
    d += part[3 * b + 1];
    const double x = part[3 * b + 2];
    r = (x > r || x != x) ? x : r;
  }
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) {
    o += __shfl_down(o, k, 64);
    d += __shfl_down(d, k, 64);
    const double x = __shfl_down(r, k, 64);
    r = (x > r || x != x) ? x : r;
  }
  if (t == 0) {
    out[0] = o;
    out[1] = d;
    out[2] = r;
  }
}

struct RefineWork {
  double2 *mat[7], *W, *gpart;
  double *lam, *lam2, *part, *norms;
  unsigned long long* emax;
  int *rank, *order, *reach, *pm, *cstart, *csize, *cslot, *info;
  int2* clist;
};

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

RefineWork carve(void* work, int m) {
  RefineWork r;
  char* p = static_cast<char*>(work);
  const size_t mm = al256(size_t(m) * m * sizeof(double2));
  for (int i = 0; i < 7; ++i) { r.mat[i] = reinterpret_cast<double2*>(p); p += mm; }
  r.W = reinterpret_cast<double2*>(p);
  p += al256(size_t(m / 2 + 1) * KMAX * KMAX * sizeof(double2));
  auto dbl = [&](size_t n) { double* q = reinterpret_cast<double*>(p); p += al256(n * sizeof(double)); return q; };
  auto in = [&](size_t n) { int* q = reinterpret_cast<int*>(p); p += al256(n * sizeof(int)); return q; };
  r.lam = dbl(m);
  r.lam2 = dbl(m);
  r.part = dbl(3 * CHECK_BLOCKS);
  r.norms = dbl(8);   // [0..2] check norms, [4] noise floor tau
  r.emax = reinterpret_cast<unsigned long long*>(dbl(1));
  r.rank = in(m);
  r.order = in(m);
  r.reach = in(m);
  r.pm = in(m);
  r.cstart = in(m);
  r.csize = in(m);
  r.cslot = in(m);
  r.info = in(4);
  r.clist = reinterpret_cast<int2*>(p);
  p += al256(size_t(m) * sizeof(int2));
  r.gpart = reinterpret_cast<double2*>(p);
  p += al256(gemm_square_scratch_bytes(m));
  return r;
}
}  // namespace

size_t refine_scratch_bytes(int m) {
  RefineWork r = carve(nullptr, m);
  return size_t(reinterpret_cast<char*>(r.gpart)) + al256(gemm_square_scratch_bytes(m));
}

int refine_eigh(const void* Av, int m, double* w, void* Z, void* work, const RefineTargets& tg,
                int maxit, hipStream_t st, int sq_split) {
  if (m <= 0) return 0;
  const double tol = tg.tol, noise = tg.noise, orth = tg.orth;
  RefineWork r = carve(work, m);
  const double2* A = static_cast<const double2*>(Av);
  double2 *X = r.mat[0], *Xn = r.mat[1], *Q = r.mat[2], *T = r.mat[3], *S = r.mat[4],
          *R = r.mat[5], *E = r.mat[6];
  const unsigned gm = unsigned((m + 255) / 256);
  const size_t mm = size_t(m) * m;
  const unsigned ncheck = unsigned(std::min<size_t>(CHECK_BLOCKS, (mm + 255) / 256));
  Clusters cl{r.order, r.cstart, r.csize, r.cslot, r.W};
  // noise floor of H': couplings at or below tau (noise x the rms eigenvalue)
  // are indistinguishable from the rounding of the products that formed H'
  // (8 ulps in FP64; the split-FP16 subspace matrices carry ~2^-22 of their
  // largest entries): they form no clusters, get only the orthonormality
  // term and count as converged.  The residual of the outer iteration then
  // levels off near tau times the square root of the couplings per state,
  // which is where the precision ladder hands over to FP64.
  double* tau = r.norms + 4;   // on the device: no read-back needed
  hipLaunchKernelGGL(k_ref_diag2, dim3(1), dim3(256), 0, st, A, m, noise, tau, g_launch_gate);
  for (int it = 0;; ++it) {
    const double2* Sp = A;
    const double2* Rp = nullptr;
    if (it > 0) {
      gemm_square(X, 1, X, 0, R, m, st, r.gpart, 1, sq_split);
      gemm_square(A, 0, X, 0, T, m, st, r.gpart, 0, sq_split);
      gemm_square(X, 1, T, 0, S, m, st, r.gpart, 1, sq_split);
      hipLaunchKernelGGL(k_ref_check, dim3(ncheck), dim3(256), 0, st, S, R, m, (const double*)tau,
                         r.part, g_launch_gate);
      hipLaunchKernelGGL(k_ref_check_final, dim3(1), dim3(64), 0, st, (const double*)r.part,
                         int(ncheck), r.norms, g_launch_gate);
      double h[3];
      int hi[2];
      hipMemcpyAsync(h, r.norms, sizeof(h), hipMemcpyDeviceToHost, st);
      hipMemcpyAsync(hi, r.info, sizeof(hi), hipMemcpyDeviceToHost, st);
      hipStreamSynchronize(st);
      if (!(h[0] == h[0]) || !(h[1] == h[1]) || !(h[2] == h[2]) || hi[1] > KMAX) return -1;
      if ((h[0] <= tol * tol * h[1] || h[0] < 1e-300) && h[2] <= orth) {
        eig_sort(S, X, m, m, w, Z, st);
        return it;
      }
      if (it >= maxit) return -1;
      Sp = S;
      Rp = R;
      hipLaunchKernelGGL(k_ref_tau, dim3(1), dim3(64), 0, st, (const double*)r.norms, m, noise, tau, g_launch_gate);
    }
    hipLaunchKernelGGL(k_ref_lambda, dim3(gm), dim3(256), 0, st, Sp, Rp, m, r.lam, r.emax, g_launch_gate);
    hipLaunchKernelGGL(k_ref_rank, dim3((m + 63) / 64), dim3(64 * RANK_SPLIT), 0, st, (const double*)r.lam, m, r.rank, r.order, g_launch_gate);
    hipLaunchKernelGGL(k_ref_reach, dim3(m), dim3(256), 0, st, Sp, Rp, (const double*)r.lam,
                       (const int*)r.rank, m, THETA, (const double*)tau, r.reach, g_launch_gate);
    hipLaunchKernelGGL(k_ref_clusters, dim3(1), dim3(1024), 0, st, (const int*)r.reach, m, r.pm,
                       r.cstart, r.csize, r.cslot, r.clist, r.info, g_launch_gate);
    hipLaunchKernelGGL(k_ref_cluster_eig, dim3(unsigned(m / 2 + 1)), dim3(256), 0, st, Sp, Rp, m,
                       (const int*)r.order, (const int2*)r.clist, (const int*)r.info, r.W, tol * 1e-2, g_launch_gate);
    hipLaunchKernelGGL(k_ref_lambda2, dim3(gm), dim3(256), 0, st, Sp, Rp, m, cl, r.lam2, g_launch_gate);
    ref_update(Sp, Rp, m, cl, r.lam2, tau, E, r.emax, st);
    // E^2/2 only while |E| > e2skip, decided on the device (as in the
    // device-decided refinement, so that the two take the same arithmetic)
    int* e2 = r.info + 3;
    hipLaunchKernelGGL(k_ref_e2_flag, dim3(1), dim3(64), 0, st, (const unsigned long long*)r.emax,
                       g_launch_gate, tg.e2skip, e2);
    {
      GateScope g2(e2);
      gemm_square(E, 0, E, 0, T, m, st, r.gpart, 0, sq_split);
    }
    hipLaunchKernelGGL(k_ref_build_q, dim3(gm, unsigned(m)), dim3(256), 0, st, (const double2*)E,
                       (const double2*)T, (const int*)e2, m, cl, Q, g_launch_gate);
    if (it == 0) {
      std::swap(X, Q);
    } else {
      gemm_square(X, 0, Q, 0, Xn, m, st, r.gpart, 0, sq_split);
      std::swap(X, Xn);
    }
  }
}

// ------------------------------------------------------------------ device-decided
// The stop test of refine_eigh on the device (ungated; one thread).
__global__ void k_ref_decide(const double* __restrict__ norms, const int* __restrict__ info,
                             double tol, double orth, int it, int maxit, int* __restrict__ flags,
                             int set) {
  if (threadIdx.x != 0) return;
  if (flags[F_REF_RUN] == 0) {
    flags[F_REF_OK + it] = 0;
    return;
  }
  const double h0 = norms[0], h1 = norms[1], h2 = norms[2];
  flags[F_REF_STEPS] = it;
  const bool bad = !(h0 == h0) || !(h1 == h1) || !(h2 == h2) || info[1] > KMAX;
  const bool conv = !bad && (h0 <= tol * tol * h1 || h0 < 1e-300) && h2 <= orth;
  flags[F_REF_OK + it] = conv ? 1 : 0;
  if (conv) {
    flags[F_REF_RUN] = 0;
  } else if (bad || it >= maxit) {
    flags[F_REF_RUN] = 0;
    flags[F_HOST] = HOST_REFINE;
    flags[F_HOST_SET] = set;
    flags[F_ACTIVE] = 0;
  }
}

__global__ void k_ref_start(int* __restrict__ flags) {
  if (threadIdx.x != 0) return;
  flags[F_REF_RUN] = flags[F_ACTIVE];
  flags[F_REF_STEPS] = 0;
}

void refine_eigh_dev(const void* Av, int m, double* w, void* Z, void* work, const RefineTargets& tg,
                     int maxit, hipStream_t st, int sq_split, int* flags, int set) {
  if (m <= 0) return;
  const double tol = tg.tol, noise = tg.noise, orth = tg.orth;
  if (maxit > F_NFLAGS - F_REF_OK - 1) maxit = F_NFLAGS - F_REF_OK - 1;
  RefineWork r = carve(work, m);
  const double2* A = static_cast<const double2*>(Av);
  double2 *X = r.mat[0], *Xn = r.mat[1], *Q = r.mat[2], *T = r.mat[3], *S = r.mat[4],
          *R = r.mat[5], *E = r.mat[6];
  const unsigned gm = unsigned((m + 255) / 256);
  const size_t mm = size_t(m) * m;
  const unsigned ncheck = unsigned(std::min<size_t>(CHECK_BLOCKS, (mm + 255) / 256));
  Clusters cl{r.order, r.cstart, r.csize, r.cslot, r.W};
  double* tau = r.norms + 4;
  const int* run = flags + F_REF_RUN;
  hipLaunchKernelGGL(k_ref_start, dim3(1), dim3(64), 0, st, flags);
  {
    GateScope g(run);
    hipLaunchKernelGGL(k_ref_diag2, dim3(1), dim3(256), 0, st, A, m, noise, tau, g_launch_gate);
  }
  for (int it = 0; it <= maxit; ++it) {
    const double2* Sp = A;
    const double2* Rp = nullptr;
    if (it > 0) {
      {
        GateScope g(run);
        gemm_square(X, 1, X, 0, R, m, st, r.gpart, 1, sq_split);
        gemm_square(A, 0, X, 0, T, m, st, r.gpart, 0, sq_split);
        gemm_square(X, 1, T, 0, S, m, st, r.gpart, 1, sq_split);
        hipLaunchKernelGGL(k_ref_check, dim3(ncheck), dim3(256), 0, st, S, R, m, (const double*)tau,
                           r.part, g_launch_gate);
        hipLaunchKernelGGL(k_ref_check_final, dim3(1), dim3(64), 0, st, (const double*)r.part,
                           int(ncheck), r.norms, g_launch_gate);
      }
      hipLaunchKernelGGL(k_ref_decide, dim3(1), dim3(64), 0, st, (const double*)r.norms,
                         (const int*)r.info, tol, orth, it, maxit, flags, set);
      {
        GateScope g(flags + F_REF_OK + it);
        eig_sort(S, X, m, m, w, Z, st);
      }
      if (it == maxit) break;
      Sp = S;
      Rp = R;
      GateScope g(run);
      hipLaunchKernelGGL(k_ref_tau, dim3(1), dim3(64), 0, st, (const double*)r.norms, m, noise, tau,
                         g_launch_gate);
    }
    GateScope g(run);
    hipLaunchKernelGGL(k_ref_lambda, dim3(gm), dim3(256), 0, st, Sp, Rp, m, r.lam, r.emax, g_launch_gate);
    hipLaunchKernelGGL(k_ref_rank, dim3((m + 63) / 64), dim3(64 * RANK_SPLIT), 0, st, (const double*)r.lam, m, r.rank,
                       r.order, g_launch_gate);
    hipLaunchKernelGGL(k_ref_reach, dim3(m), dim3(256), 0, st, Sp, Rp, (const double*)r.lam,
                       (const int*)r.rank, m, THETA, (const double*)tau, r.reach, g_launch_gate);
    hipLaunchKernelGGL(k_ref_clusters, dim3(1), dim3(1024), 0, st, (const int*)r.reach, m, r.pm,
                       r.cstart, r.csize, r.cslot, r.clist, r.info, g_launch_gate);
    hipLaunchKernelGGL(k_ref_cluster_eig, dim3(unsigned(m / 2 + 1)), dim3(256), 0, st, Sp, Rp, m,
                       (const int*)r.order, (const int2*)r.clist, (const int*)r.info, r.W,
                       tol * 1e-2, g_launch_gate);
    hipLaunchKernelGGL(k_ref_lambda2, dim3(gm), dim3(256), 0, st, Sp, Rp, m, cl, r.lam2, g_launch_gate);
    ref_update(Sp, Rp, m, cl, r.lam2, tau, E, r.emax, st);
    int* e2 = r.info + 3;
    hipLaunchKernelGGL(k_ref_e2_flag, dim3(1), dim3(64), 0, st, (const unsigned long long*)r.emax,
                       run, tg.e2skip, e2);
    {
      GateScope g2(e2);
      gemm_square(E, 0, E, 0, T, m, st, r.gpart, 0, sq_split);
    }
    hipLaunchKernelGGL(k_ref_build_q, dim3(gm, unsigned(m)), dim3(256), 0, st, (const double2*)E,
                       (const double2*)T, (const int*)e2, m, cl, Q, g_launch_gate);
    if (it == 0) {
      std::swap(X, Q);
    } else {
      gemm_square(X, 0, Q, 0, Xn, m, st, r.gpart, 0, sq_split);
      std::swap(X, Xn);
    }
  }
}

}  // namespace sky
