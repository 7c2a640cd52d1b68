// Host-side launchers of the library's kernels (all enqueue on `st`).
#pragma once

#include <string>

#include "sky_common.h"

namespace sky {

// ---- launch gate
// Every kernel of the library takes a gate: a device int that it reads first,
// returning at once if it is 0 (nullptr: always run).  The launchers pass the
// calling thread's current gate, nullptr unless a GateScope is open, so that
// a context can mask a box's kernels, or pick between branches of its
// iteration, from values computed on the device (a captured iteration then
// needs no host decision).
extern thread_local const int* g_launch_gate;
struct GateScope {
  const int* prev;
  explicit GateScope(const int* g) : prev(g_launch_gate) { g_launch_gate = g; }
  ~GateScope() { g_launch_gate = prev; }
  GateScope(const GateScope&) = delete;
  GateScope& operator=(const GateScope&) = delete;
};

// ---- device-decided iteration: flags of one box (ints in device memory)
// F_ACTIVE: the box's iteration kernels run (cleared at convergence, or
//   when a decision needs the host); F_HOST: 0, or the stage that stopped
//   the box (HOST_LOEWDIN: the overlap is too far from the identity for the
//   series, or not finite; HOST_REFINE: the refinement did not converge;
//   HOST_NAN: a non-finite residual) and F_HOST_SET its state set;
//   F_ITER: iterations completed on the device; F_CONV: Delta-eps <= tol;
//   F_SERIES + k: Horner step k of the Loewdin series runs; F_REF_RUN: the
//   refinement continues; F_REF_OK + it: it converged at check it (its
//   eigenpairs are sorted out there); F_REF_STEPS: refinement steps taken.
enum DevFlag {
  F_ACTIVE = 0, F_HOST = 1, F_HOST_SET = 2, F_ITER = 3, F_CONV = 4, F_REF_RUN = 5,
  F_REF_STEPS = 6, F_SERIES = 8, F_REF_OK = 24, F_NFLAGS = 64
};
enum HostStage { HOST_NONE = 0, HOST_LOEWDIN = 1, HOST_REFINE = 2, HOST_NAN = 3 };
// doubles beside the flags: D_TOL (the tolerance), D_DE (the last Delta-eps),
// D_SERIES.. (norm, term count and the series coefficients of the last solve)
enum DevDouble { D_TOL = 0, D_DE = 1, D_SERIES = 4, D_NDOUBLES = 32 };
void set_flag(int* flags, int idx, int value, hipStream_t st);   // ungated
void set_double(double* d, int idx, double value, hipStream_t st);   // ungated

// ---- grid kernels (k_grid.hip); states are [state][2][n^3], complex128
// (prec 0) or complex64 (prec 1); reductions are FP64 either way.
int grid_ntiles(int n);  // room for the per-state partials of one pass
// lines: 0 = default; H_PLANE = z by line pencils, x and y on LDS z-slices;
// else pencils per workgroup of the three line passes.  h_pass_lines fills
// the supported values (out[4]) and returns their count; h_pass_default is
// what 0 selects.  apply_h returns 0 if lines is not supported.
constexpr int H_PLANE = -1;
int h_pass_lines(int n, int prec, int* out);
int h_pass_default(int n, int prec);
// 1 if the damped step has the LDS-slice variant on this grid and precision.
int damp_slices_available(int n, int prec);
// amax (optional): the largest |component| of h psi is merged into it (float
// bits; clear it first), as plane_scale would compute it.
int apply_h(int n, int prec, const void* psi, void* hpsi, int nstate, MeanFieldPtrs mf,
            GridArgs g, double* eps_part, double* eps, hipStream_t st, int lines = 0,
            unsigned int* amax = nullptr);
// gain (optional, [state][PC_SHELLS]): multiplies the damping per |k| shell.
// shell_pow (optional, [state][PC_SHELLS], accumulated: clear first): the
// residual's spectral power per shell, from an extra read-only pass.
// xy: 1 = x and y transforms on LDS z-slices where they fit, 0 = line
// passes, -1 = the default for the grid and precision.  amax (optional):
// the largest |component| of phi is merged into it (stages 0 and 2).
// stage 0: whole step; 1: up to the shell powers (partial spectrum left in
// phi, r2 formed); 2: the rest, continuing from stage 1 (gains decided in
// between).
void damped_step(int n, int prec, const void* psi, const void* hpsi, const double* eps,
                 void* phi, int nstate, GridArgs g, double x0, double e0, double hb2m,
                 double* r2_part, double* r2, hipStream_t st, const float* gain = nullptr,
                 double* shell_pow = nullptr, int stage = 0, int xy = -1,
                 unsigned int* amax = nullptr);

// ---- learned preconditioner (k_precond.hip)
int precond_nparams();
int precond_ns_max();
void precond_init_params(float* P_dev, unsigned seed, hipStream_t st);
void precond_round(const float* P, float* Pb, hipStream_t st);
void precond_forward(const float* Pb, const float* X, int B, float* H1, float* H2, float* H3,
                     float* O, hipStream_t st);
// rows [a*S + s][6] = (features, target, weight) of states a < ns; pow and eps
// rows of state a at a*stride
void precond_features(const double* pow, const double* eps, int stride, int ns, double e0,
                      double hb2m, double kmax, float* X, hipStream_t st);
void precond_gains(const float* O, int n, float* gain, hipStream_t st);
// loss and parameter gradient G; gpart: precond_gpart_bytes(B) of chunk
// partials of G; dscratch >= B/256 + 2 doubles; want_loss: synchronise and
// return the loss (else 0).
double precond_loss_grad(const float* Pb, const float* S, int B, double wsum, float* H1,
                         float* H2, float* H3, float* O, float* dO, float* D1, float* D2,
                         float* D3, float* G, float* gpart, double* dscratch, int want_loss,
                         hipStream_t st);
size_t precond_gpart_bytes(int rows);
void precond_adam(float* P, const float* G, float* M, float* V, int step, float lr,
                  hipStream_t st);
void precond_gather(int prec, const void* psi, const void* hpsi, const double* eps,
                    const int* idx, int ns, long V, void* bpsi, void* bh, double* beps,
                    float* onehot, hipStream_t st);
void precond_dir(int prec, const void* bpsi, void* bphi, size_t n, hipStream_t st);
size_t precond_gram_bytes(int ns);
void precond_targets(int prec, const void* bpsi, const void* bh, const void* bd, const void* bhd,
                     const double* beps, int ns, long V, double* part, float* S, hipStream_t st);
// dens = 11 fields [rho, tau, Jx, Jy, Jz, sx, sy, sz, jx, jy, jz][n^3],
// summed over the first nstate states of each of ngroup state arrays psi[t]
// (each with its own grid arguments g[t], i.e. its twist; spacing from g[0])
// and divided by ngroup (the twist average); part holds nchunk_max * 16 * n^3
// doubles.  Returns 0 (nothing launched) for ngroup outside [0,
// DENS_MAX_GROUPS] or nchunk_max < 1.
constexpr int DENS_MAX_GROUPS = 32;
struct DensGroups {
  const void* psi[DENS_MAX_GROUPS];
  double kshift[DENS_MAX_GROUPS][3];   // GridArgs::tw of each group
  int ngroup;
};
int densities(int n, int prec, const void* const* psi, const GridArgs* g, int ngroup,
               int nstate, int nchunk_max, double* part, double* dens, hipStream_t st);
// n complex values between precisions (0 = complex128, 1 = complex64).
void convert_states(const void* src, int src_prec, void* dst, int dst_prec, size_t n,
                    hipStream_t st);

// ---- allocation-free scratch (k_noalloc.hip): a fixed device array per
// device; noalloc_scratch returns its address on the current device (looked
// up once per device), or -1 with a message.
size_t noalloc_scratch_capacity();   // doubles
int noalloc_scratch(double** ptr, std::string* err);

// ---- mean field and energy (k_fields.hip)
struct Skyrme {
  double b0, b0p, b1, b1p, b2, b2p, b3, b3p, b4, b4p, alpha;
  double hb2m_n, hb2m_p, e2;
};
// dens[q] as produced by densities(); derived[q] = 5 fields [lap rho, d rho (3), div J];
// mf[q] = 5 fields [U, B, Wx, Wy, Wz]; vc = Coulomb potential;
// scratch >= 2 n^3 complex + 4 n doubles (mean_field_scratch_bytes).
// epart: per-block energy partials, energy[8] = {kin, rho, rho3, tau, lap, so, coul, total}.
void mean_field(int n, GridArgs g, const Skyrme& sk, const double* dens_n,
                const double* dens_p, double* derived_n, double* derived_p, double* mf_n,
                double* mf_p, double* vc, void* scratch, double* epart, double* energy,
                hipStream_t st);
int energy_nblocks(int n);
size_t mean_field_scratch_bytes(int n);

// ---- dense complex matrices (k_gemm.hip); complex128, row-major
// C[a][b] = scale * sum_v conj(A[a][v]) B[b][v] for b <= a (lower triangle),
// for two right operands at once (B0 -> C0, B1 -> C1, B1 may be null).
// part: split * 2 * ntile_pairs * 64*64 complex scratch.
size_t overlap_scratch_bytes(int m, long k);
// ev (may be null): events recorded right before / after the GEMM kernel.
// split_req > 0 overrides the split-K factor (one of overlap_split_candidates).
int overlap_split_candidates(int m, long k, int* out);
void overlap_lower(const void* A, const void* B0, const void* B1, int m, long k, double scale,
                   void* C0, void* C1, void* part, hipStream_t st, hipEvent_t* ev = nullptr,
                   int split_req = 0);
// FP64 reduction of split-K partials into the lower tiles of C0 (and C1).
void overlap_reduce(const void* part, int npair, int split, int m, double scale, void* C0,
                    void* C1, int nz, hipStream_t st);
// Mixed precision (k_gemm_mixed.hip): complex64 operands split once into
// FP16 planes (re h, re l, im h, im l; 8 bytes per complex) under a
// power-of-two scale per matrix, FP16 MFMA with FP32 accumulation folded into
// FP64.  plane_scale writes the bit pattern of the largest |component| of x
// (n complex values) to *mx; the split and product calls read it there.
// NT planes hold a rows x k matrix as [4][rows][k]; transposed planes of a
// rows x cols matrix hold [4][cols][planes_pad(rows)] (zero-padded).
size_t overlap_scratch_bytes_mixed(int m, long k);
long planes_pad(int m);
size_t planes_bytes_nt(int rows, long k);
size_t planes_bytes_t(int m, long cols);
// The plane products' direct tile loads address a 128-row tile with 32-bit
// byte offsets below 2^31: true for every grid of 64^3 or less with at most
// 2 n^3 states.
bool planes_direct_ok(int m, long k);
void plane_scale(const void* x, int x_is_c128, size_t n, unsigned int* mx, hipStream_t st);
// Zero n largest-|component| slots (before producers merge into them).
void clear_scales(unsigned int* mx, int n, hipStream_t st);
void split_planes_nt(const void* x, int rows, long k, const unsigned int* mx, void* P,
                     hipStream_t st);
void split_planes_t(const void* x, int x_is_c128, int rows, long cols, const unsigned int* mx,
                    void* P, hipStream_t st);
// split_planes_nt into P and split_planes_t into PT of the same complex64
// matrix (rows x k) from one read of it.
void split_planes_both(const void* x, int rows, long k, const unsigned int* mx, void* P, void* PT,
                       hipStream_t st);
// C0 = scale * conj(A) B0^T (and C1 with B1), lower 64-tiles, from NT planes.
// split_req > 0 overrides the split-K factor (one of overlap_split_candidates_mixed).
int overlap_split_candidates_mixed(int m, long k, int* out);
void overlap_lower_planes(const void* PA, const void* PB0, const void* PB1,
                          const unsigned int* mxA, const unsigned int* mxB0,
                          const unsigned int* mxB1, int m, long k, double scale, void* C0,
                          void* C1, void* part, hipStream_t st, hipEvent_t* ev = nullptr,
                          int split_req = 0, int waves = 8);
// Y[b][v] = sum_a U[a][b] X[a][v] from the transposed planes of U (m x m)
// and of X (m x k).  waves, for both plane products: 8 (32 x 64 per wave)
// or 4 (64 x 64 per wave) per 128 x 128 output tile; both load their tiles
// straight into two alternating LDS buffers (128 KB of LDS per workgroup),
// which needs planes_direct_ok(m, k).
void combine_planes(const void* PU, const void* PX, const unsigned int* mxU,
                    const unsigned int* mxX, void* Y, int m, long k, hipStream_t st,
                    int waves = 8);
// Fill the upper triangle of Hermitian C from the lower one (and make the
// diagonal real), in place.
void hermitian_fill(void* C, int m, hipStream_t st);
// Y[b][v] = sum_a U[a][b] X[a][v]   (psi = phi U), X: m x k, U: m x m (ld m)
void combine(const void* X, const void* U, void* Y, int m, long k, hipStream_t st);
// C = op(A) op(B), square m x m; opA/opB: 0 = N, 1 = conjugate transpose.
// With part (>= gemm_square_scratch_bytes(m)) the contraction is split over
// more workgroups and the FP64 partials are summed in a fixed order.  herm:
// the product is known to be Hermitian; only its lower tiles are computed and
// the upper triangle is mirrored from them (C exactly Hermitian).
size_t gemm_square_scratch_bytes(int m);
// split_req > 0 overrides the split-K factor (one of square_split_candidates).
int square_split_candidates(int m, int* out);
void gemm_square(const void* A, int opA, const void* B, int opB, void* C, int m, hipStream_t st,
                 void* part = nullptr, int herm = 0, int split_req = 0);

// ---- eigenvector refinement (k_refine.hip)
// Hermitian eigen-decomposition of a nearly diagonal A (m x m, not modified)
// by Newton-type refinement with exact solves of near-degenerate clusters:
// w ascending, Z columns.  Returns the refinement steps taken, or -1 when it
// cannot finish (a cluster wider than its limit, a non-finite value, or more
// than maxit steps); the caller then uses jacobi_eigh.  Converged when the
// relative off-diagonal Frobenius norm of Z^H A Z is below tol and
// max |Z^H Z - 1| below orth.  noise: the relative precision of A's entries
// (x its rms eigenvalue = the coupling floor below which entries are noise:
// no clusters, no rotation, counted as converged); 8 ulps for A from FP64
// products.  Synchronises the stream once per step.
size_t refine_scratch_bytes(int m);
// Stop and step targets of the refinement.
struct RefineTargets {
  double tol;      // relative off-diagonal Frobenius norm of Z^H A Z at convergence
  double noise;    // relative precision of A's entries (see above)
  double orth;     // max |Z^H Z - 1| at convergence
  double e2skip;   // an update forms its E^2/2 term while max |E| > e2skip
};
int refine_eigh(const void* A, int m, double* w, void* Z, void* work, const RefineTargets& tg,
                int maxit, hipStream_t st, int sq_split = 0);
// The same refinement with its decisions on the device (launches only): up
// to maxit steps, each gated by flags[F_REF_RUN]; the check after step it
// sorts the eigenpairs out when converged (flags[F_REF_OK + it]); a step
// that would make the host version give up (maxit reached, a cluster over
// the limit, a non-finite check) sets F_HOST = HOST_REFINE (set `set`) and
// clears F_ACTIVE.  The E^2 term of the update is always formed.  maxit <=
// F_NFLAGS - F_REF_OK - 1.
void refine_eigh_dev(const void* A, int m, double* w, void* Z, void* work, const RefineTargets& tg,
                     int maxit, hipStream_t st, int sq_split, int* flags, int set);

// ---- dense FP64 linear algebra (k_linalg.hip)
// Cholesky A = L L^H of Hermitian positive definite A (m x m, lower used),
// then Linv = L^-1 (lower triangular, upper zeroed).  info[0] != 0 when a
// pivot is not above piv_min (or not a number).  work >= m*m complex.
void cholesky_inverse(void* A, void* Linv, int m, void* work, int* info, hipStream_t st,
                      double piv_min = 0.0);
// Hermitian eigen-decomposition by blocked two-sided Jacobi: A (m x m, full
// Hermitian, destroyed) -> eigenvalues w (ascending) and eigenvectors Z
// (columns).  work: jacobi_scratch_bytes(m).
// Returns the sweeps taken, -1 when the off-diagonal norm is still above tol
// after max_sweeps sweeps (w, Z then hold the last sweep's result), -2 when
// the matrix holds a non-finite value.
size_t jacobi_scratch_bytes(int m);
int jacobi_eigh(void* A, int m, double* w, void* Z, void* work, double tol, int max_sweeps,
                hipStream_t st);
// Gauge of the paper-literal update: info[3c..3c+2] = (start, size, packed
// offset) of the eigenvalue cluster of column c.  gauge_gather packs each
// cluster's diagonal block of Z (row-major, m x m); gauge_apply writes
// out = Z Q for the block-diagonal Q whose blocks are packed the same way.
void gauge_gather(const void* Z, int m, const int* info, void* packed, hipStream_t st);
void gauge_apply(const void* Z, int m, const int* info, const void* Q, void* out, hipStream_t st);
// Loewdin transform C = I^-1/2 (Eqs. Loewedin/orthmatvec) of an overlap close
// to the identity, by the binomial series of (1 + D)^-1/2, D = I - 1, in
// Horner form on the FP64 matrix cores.  The number of terms p makes the
// remainder (bounded through ||D||_2 <= ||D||_F) smaller than eps.
// Returns p, 0 (nothing written to C) when ||D||_F > max_dev, or -1 when
// ||D||_F is not a finite number.  D and T
// are m x m work matrices, scratch >= 257 doubles, part the square-product
// scratch (gemm_square); synchronises the stream.
int loewdin_series(const void* I, void* C, void* D, void* T, int m, double max_dev,
                   double* scratch, void* part, hipStream_t st, int sq_split = 0, double eps = 0x1p-56);
// The series with the decision on the device: the term count from the norm
// of D = I - 1 (as loewdin_series), Horner steps gated by flags[F_SERIES + k].
// If the series does not apply (norm above max_dev or not finite), flags
// get F_HOST = HOST_LOEWDIN (set `set`) and F_ACTIVE = 0.  dbl: the box's
// doubles (D_SERIES..).  Launches only.
void loewdin_series_dev(const void* I, void* C, void* D, void* T, int m, double max_dev,
                        double eps, double* scratch, void* part, hipStream_t st, int sq_split,
                        int* flags, double* dbl, int set);
// End of a device-decided iteration (one workgroup, ungated): if the box is
// active, F_ITER += 1 and Delta-eps = sqrt(sum of ||r||^2 over the first
// nocc[s] states of each set s / count) goes to dbl[D_DE]; Delta-eps <=
// dbl[D_TOL] sets F_CONV and clears F_ACTIVE; a non-finite one sets
// F_HOST = HOST_NAN.  Up to 64 sets.
void iteration_end(const double* const* r2, const int* nocc, int nset, int count, int* flags,
                   double* dbl, hipStream_t st);
// w ascending (ties by index) from the diagonal of D (ld = ld) and Z the
// matching columns of V (ld = ld), Z m x m.
void eig_sort(const void* D, const void* V, int m, int ld, double* w, void* Z, hipStream_t st);
// X <- X diag(d) (scale column b by d[b]), d real.
void scale_columns(void* X, const double* d, int m, hipStream_t st);
// w <- w^-1/2 elementwise (Loewdin), flags info if any w <= floor_v.
void inv_sqrt(double* w, int m, int* info, hipStream_t st, double floor_v = 0.0);
// fill n doubles (floats) with zero (a kernel, so it can be captured in graphs)
void zero(double* p, size_t n, hipStream_t st);
void zero_f32(float* p, size_t n, hipStream_t st);
// A = the m x m unit matrix (complex128).
void identity(void* A, int m, hipStream_t st);

}  // namespace sky
