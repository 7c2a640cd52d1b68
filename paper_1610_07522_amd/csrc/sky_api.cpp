// C ABI of the damped-gradient solver: context, workspace layout and the
// static iteration of Fig. 1 (steps 2-5) of the paper.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sky.h"
#include "sky_kernels.h"

using namespace sky;

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return SKY_OK;
  return fail(SKY_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool grid_ok(int n) {
  return n == 8 || n == 16 || n == 24 || n == 32 || n == 48 || n == 64;
}

constexpr size_t ALIGN = 256;
size_t al(size_t b) { return (b + ALIGN - 1) / ALIGN * ALIGN; }

constexpr int MAXSET = 2 * SKY_MAX_TWIST;   // state sets: species x twists
constexpr int DENS_CHUNKS = 32;   // state chunks of the density passes
static_assert(SKY_MAX_TWIST <= sky::DENS_MAX_GROUPS, "one density launch covers every twist");
constexpr int PC_CAP = 16384;     // sample rows of the learned preconditioner
constexpr int PC_HOLD = 10;       // iterations on plain damping after a rise of the residual
constexpr int PC_RETRAIN_STEPS = 20;   // Adam steps of each online training
constexpr double JACOBI_TOL = 1e-12;   // relative off-diagonal Frobenius norm
constexpr int JACOBI_SWEEPS = 30;
constexpr int REFINE_ITERS = 10;     // refinement steps before the Jacobi fallback
// refinement steps of the device-decided iteration before it hands the set
// to the host path (which takes up to REFINE_ITERS, then Jacobi)
constexpr int REFINE_ITERS_DEV = 4;
// ||I - 1||_F up to which I^-1/2 comes from its binomial series (<= 8 terms)
constexpr double LOEWDIN_SERIES_MAX = 1e-2;
// relative precision of H' built from the split-FP16 overlap and Hamiltonian
// matrices (their representation error is 2^-22 of the largest entries; x2)
constexpr double MIXED_HP_NOISE = 0x1p-21;
// targets of the eigenvector refinement (off-diagonal norm, noise floor of
// H', max |Z^H Z - 1|, smallest |E| whose E^2/2 term is formed): FP64, and
// the mixed form, whose U is rounded to the split-FP16 planes (2^-22
// relative) by the recombination and whose states are stored in complex64
// (2^-24): a Z orthonormal beyond 2^-30 would be rounded away there, and an
// E^2/2 below 2^-33 is an eighth of that target
const RefineTargets REFINE_FP64{JACOBI_TOL, 0x1p-49, 1e-13, 1e-8};
const RefineTargets REFINE_MIXED{JACOBI_TOL, MIXED_HP_NOISE, 0x1p-30, 0x1p-16};
// truncation bound of the Loewdin series (remainder of C = I^-1/2): FP64,
// and the mixed form, an order of magnitude below its orthonormality target
constexpr double SERIES_EPS = 0x1p-56;
constexpr double MIXED_SERIES_EPS = 0x1p-34;
// smallest Cholesky pivot (or overlap eigenvalue, for Loewdin) of an
// overlap matrix (unit diagonal): below it the states are linearly
// dependent for any practical purpose
constexpr double CHOL_PIVOT_MIN = 1e-10;
// paper-literal update: eigenvalues of H closer than this (MeV) form one
// cluster of the gauge of Z
constexpr double PAPER_CLUSTER_TOL = 1e-3;

// Byte offsets of every buffer inside the caller's workspace.
struct Layout {
  // per state set (species x twist): complex128 states, complex64 copies
  // (mixed only), Rayleigh quotients, residuals, subspace eigenvalues
  size_t psi[MAXSET], hpsi[MAXSET], psi32[MAXSET], hpsi32[MAXSET];
  size_t eps[MAXSET], r2[MAXSET], ritz[MAXSET];
  // per species, shared by its twists (one set is in flight at a time)
  size_t phi[2], hphi[2], phi32[2], hphi32[2];
  size_t tiles, gauge;
  size_t matI, matH, matC, matL, matT, matHp, matZ, matU, wtmp, gemm_part, chol_work, jac_work;
  size_t ref_work, nrm, sq_part;
  // learned preconditioner: parameters (FP32 master, BF16-rounded copy),
  // gradient, Adam moments, sample rows, activations, shell powers, gains,
  // sampled-state batch buffers
  size_t pc_P, pc_Pb, pc_G, pc_M, pc_V, pc_S, pc_H[3], pc_D[3], pc_O, pc_dO, pc_X, pc_pow,
      pc_gain, pc_dscr, pc_gram, pc_idx, pc_beps, pc_b[4], pc_gpart;
  int pc_nb;   // largest sampled-state batch (states x shells)
  size_t plA, plB, plT, plU, plS;                  // FP16 split planes, scales (mixed only)
  size_t dens[2], der[2], mf[2], mf32[2], vc, fscratch, dens_part, epart, energy, info;
  size_t gflags, gdbl;   // flags and doubles of the device-decided iteration
  size_t total;
};

int ntwist_of(const sky_box_desc& d) { return std::max(1, d.ntwist); }
// states per set of species q: its particles plus its extra states
int states_of(const sky_box_desc& d, int q) {
  return q ? d.n_protons + d.extra_p : d.n_neutrons + d.extra_n;
}

Layout plan(const sky_box_desc& d) {
  Layout L{};
  const size_t n3 = size_t(d.n) * d.n * d.n;
  const size_t V = 2 * n3;
  const int nq[2] = {states_of(d, 0), states_of(d, 1)};
  const int nset = 2 * ntwist_of(d);
  const int nmax = std::max(1, std::max(nq[0], nq[1]));
  const size_t c16 = 16;  // bytes per complex128
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += al(std::max<size_t>(bytes, 1));
    return o;
  };
  const bool mixed = d.precision == SKY_MIXED;
  for (int s = 0; s < nset; ++s) {
    const int q = s & 1;
    const size_t sb = size_t(nq[q]) * V * c16;
    L.psi[s] = take(sb);
    L.hpsi[s] = take(sb);
    const size_t sb32 = mixed ? sb / 2 : 0;
    L.psi32[s] = take(sb32);
    L.hpsi32[s] = take(sb32);
    L.eps[s] = take(sizeof(double) * nq[q]);
    L.r2[s] = take(sizeof(double) * nq[q]);
    L.ritz[s] = take(sizeof(double) * nq[q]);
  }
  for (int q = 0; q < 2; ++q) {
    const size_t sb = size_t(nq[q]) * V * c16;
    L.phi[q] = take(sb);
    L.hphi[q] = take(sb);
    const size_t sb32 = mixed ? sb / 2 : 0;
    L.phi32[q] = take(sb32);
    L.hphi32[q] = take(sb32);
  }
  L.gauge = take(sizeof(int) * 3 * size_t(nmax));
  const int ntile = grid_ntiles(d.n);
  L.pc_nb = std::min(precond_ns_max(), nmax) * PC_SHELLS;
  L.tiles = take(sizeof(double) * size_t(std::max(nmax, L.pc_nb)) * ntile);
  const size_t mm = size_t(nmax) * nmax * c16;
  L.matI = take(mm);
  L.matH = take(mm);
  L.matC = take(mm);
  L.matL = take(mm);
  L.matT = take(mm);
  L.matHp = take(mm);
  L.matZ = take(mm);
  L.matU = take(mm);
  L.wtmp = take(sizeof(double) * nmax);
  size_t gp = 0;
  for (int q = 0; q < 2; ++q) {
    gp = std::max(gp, overlap_scratch_bytes(std::max(1, nq[q]), long(V)));
    if (mixed) gp = std::max(gp, overlap_scratch_bytes_mixed(std::max(1, nq[q]), long(V)));
  }
  L.gemm_part = take(gp);
  // split planes of phi and h phi (rows = states), of phi^T and of U^T, shared
  // by both species (one species is in flight at a time)
  L.plA = take(mixed ? planes_bytes_nt(nmax, long(V)) : 0);
  L.plB = take(mixed ? planes_bytes_nt(nmax, long(V)) : 0);
  L.plT = take(mixed ? planes_bytes_t(nmax, long(V)) : 0);
  L.plU = take(mixed ? planes_bytes_t(nmax, nmax) : 0);
  L.plS = take(sizeof(unsigned int) * 4);   // largest |component| of phi, h phi, U
  L.chol_work = take(size_t((nmax + 63) / 64 + 1) * 64 * 64 * c16);
  L.jac_work = take(jacobi_scratch_bytes(nmax));
  // both species' sizes: the split-K scratch is not monotonic in the matrix size
  L.ref_work = take(std::max(refine_scratch_bytes(std::max(1, nq[0])),
                             refine_scratch_bytes(std::max(1, nq[1]))));
  L.nrm = take(sizeof(double) * 512);
  {
    const size_t np = size_t(precond_nparams());
    const size_t rows = std::max<size_t>(PC_CAP, size_t(nmax) * PC_SHELLS);
    const size_t pw = size_t(std::max(nmax, L.pc_nb)) * PC_SHELLS;
    L.pc_P = take(sizeof(float) * np);
    L.pc_Pb = take(sizeof(float) * np);
    L.pc_G = take(sizeof(float) * np);
    L.pc_M = take(sizeof(float) * np);
    L.pc_V = take(sizeof(float) * np);
    L.pc_S = take(sizeof(float) * 6 * PC_CAP);
    for (int i = 0; i < 3; ++i) L.pc_H[i] = take(sizeof(float) * 128 * size_t(PC_CAP));
    for (int i = 0; i < 3; ++i) L.pc_D[i] = take(sizeof(float) * 128 * size_t(PC_CAP));
    L.pc_O = take(sizeof(float) * rows);
    L.pc_dO = take(sizeof(float) * rows);
    L.pc_X = take(sizeof(float) * 6 * size_t(nmax) * PC_SHELLS);
    L.pc_pow = take(sizeof(double) * pw);
    L.pc_gain = take(sizeof(float) * pw);
    L.pc_dscr = take(sizeof(double) * (PC_CAP / 256 + 4));
    L.pc_gpart = take(precond_gpart_bytes(PC_CAP));
    L.pc_gram = take(precond_gram_bytes(precond_ns_max()));
    L.pc_idx = take(sizeof(int) * precond_ns_max());
    L.pc_beps = take(sizeof(double) * L.pc_nb);
    for (int i = 0; i < 4; ++i) L.pc_b[i] = take(c16 * size_t(L.pc_nb) * V);
  }
  L.sq_part = take(std::max(gemm_square_scratch_bytes(nq[0]), gemm_square_scratch_bytes(nq[1])));
  for (int q = 0; q < 2; ++q) {
    L.dens[q] = take(sizeof(double) * 11 * n3);
    L.der[q] = take(sizeof(double) * 5 * n3);
    L.mf[q] = take(sizeof(double) * 5 * n3);
    L.mf32[q] = take(sizeof(float) * 5 * n3);
  }
  L.vc = take(sizeof(double) * n3);
  L.fscratch = take(mean_field_scratch_bytes(d.n));
  L.dens_part = take(sizeof(double) * DENS_CHUNKS * 16 * n3);
  L.epart = take(sizeof(double) * 7 * size_t(energy_nblocks(d.n)));
  L.energy = take(sizeof(double) * 8);
  L.info = take(sizeof(int) * 4);
  L.gflags = take(sizeof(int) * F_NFLAGS);
  L.gdbl = take(sizeof(double) * D_NDOUBLES);
  L.total = off;
  return L;
}

int validate(const sky_box_desc* d) {
  if (!d) return fail(SKY_ERR_INVALID, "null descriptor");
  if (!grid_ok(d->n)) return fail(SKY_ERR_UNSUPPORTED_GRID, "grid size must be one of 8,16,24,32,48,64");
  if (!(d->dx > 0.0)) return fail(SKY_ERR_INVALID, "dx must be positive");
  if (d->n_neutrons < 0 || d->n_protons < 0 || d->n_neutrons + d->n_protons == 0)
    return fail(SKY_ERR_INVALID, "need at least one state");
  if (d->extra_n < 0 || d->extra_p < 0) return fail(SKY_ERR_INVALID, "negative extra states");
  if ((d->n_neutrons == 0 && d->extra_n > 0) || (d->n_protons == 0 && d->extra_p > 0))
    return fail(SKY_ERR_INVALID, "extra states of a species without particles");
  if (d->ntwist < 0 || d->ntwist > SKY_MAX_TWIST)
    return fail(SKY_ERR_INVALID, "ntwist must be 0..SKY_MAX_TWIST");
  for (int t = 0; t < std::max(1, d->ntwist); ++t)
    for (int m = 0; m < 3; ++m)
      if (!std::isfinite(d->twist[t][m])) return fail(SKY_ERR_INVALID, "non-finite twist");
  if (d->update != SKY_UPDATE_EXACT && d->update != SKY_UPDATE_PAPER)
    return fail(SKY_ERR_INVALID, "update must be SKY_UPDATE_EXACT or SKY_UPDATE_PAPER");
  if (d->one_h && d->update != SKY_UPDATE_EXACT)
    return fail(SKY_ERR_INVALID, "one_h needs SKY_UPDATE_EXACT");
  if (d->dev_refine_steps < 0 || d->dev_refine_steps > F_NFLAGS - F_REF_OK - 1)
    return fail(SKY_ERR_INVALID, "dev_refine_steps must be 0..39");
  const long V = 2L * d->n * d->n * d->n;
  if (states_of(*d, 0) > V || states_of(*d, 1) > V) return fail(SKY_ERR_INVALID, "more states than grid points");
  if (!(d->damp_e0 > 0.0)) return fail(SKY_ERR_INVALID, "damp_e0 must be positive");
  if (d->precision != SKY_FP64 && d->precision != SKY_MIXED)
    return fail(SKY_ERR_INVALID, "precision must be SKY_FP64 or SKY_MIXED");
  if (!planes_direct_ok(std::max(states_of(*d, 0), states_of(*d, 1)), V))
    return fail(SKY_ERR_INVALID, "plane products out of the direct-load range");
  return SKY_OK;
}
}  // namespace

struct sky_ctx {
  sky_box_desc d;
  Layout lay;
  char* ws;
  hipStream_t st;
  int n, n3;
  long V;
  int nq[2];           // states per set of species q (particles + extra states)
  int nocc[2];         // occupied states of species q (the first nocc of each set)
  int ntw, nset;       // twists; state sets = 2 * twists (set s: species s & 1)
  int prec;            // current: 0 = FP64 states, 1 = mixed (complex64 states)
  GridArgs g;          // untwisted grid arguments (fields, tuning)
  bool hpsi_lagged = false;   // one_h: h psi holds (h phi) U of the last update
  Skyrme sk;
  int last_sweeps;     // eigensolver iterations of the last iteration
  int fallbacks;       // refinement -> Jacobi fallbacks in the current call
  int unconverged;     // Jacobi solves of the current call stopped at the sweep limit
  // launch shapes (0 = the built-in default): h-pass lines per workgroup,
  // overlap and square-product split-K factors per species
  struct Tune {
    int lines = 0;
    int damp_xy = -1;   // -1: the default for the grid and precision
    int ovl[2] = {0, 0};
    int sq[2] = {0, 0};
    int ovw[2] = {0, 0};   // waves per tile of the mixed overlap product (0: 8)
    int cbw[2] = {0, 0};   // waves per tile of the mixed recombination (0: 8)
    int from_cache = 0;
    // the FP64 shapes a mixed box takes when the precision ladder switches:
    // the cache's FP64 entries for the box when sky_autotune saw them, else
    // the defaults
    int lines64 = 0;
    int damp64 = -1;
    int ovl64[2] = {0, 0};
  } tune;
  // learned preconditioner state
  int pc_count = 0;        // sample rows held
  int pc_wr = 0;           // next row written by a collection (ring)
  int pc_every = 0;        // iterations between online collections + training (0: none)
  int pc_since = 0;
  double pc_lr = 1e-3;     // Adam step of the last training call
  int pc_step = 0;         // Adam steps taken
  bool pc_trained = false;
  bool pc_ready = false;   // network initialised (first sky_init_box)
  bool pc_on = false;      // requested by sky_precond_use
  double pc_rise = 0.0;     // relative rise of the residual that triggers the fallback
  int pc_hold = 0;         // plain-damping iterations left after a residual rise
  bool pc_last = false;    // the previous iteration used the learned damping
  double de_prev = -1.0;   // residual of the previous iteration
  int pc_iters = 0;        // iterations of the current call with the learned damping
  // HIP graphs of the launch-only segments of an iteration (per species:
  // A plain / A learned, B; F = fields)
  // A variants: bit 0 = learned damping, bit 1 = h psi carried over (one_h)
  struct Graphs {
    bool on = false;
    int prec = -1;
    int captures = 0;
    hipGraphExec_t a[MAXSET][4] = {};
    hipGraphExec_t b[MAXSET] = {};
    hipGraphExec_t f = nullptr;
    // the whole iteration with its decisions on the device (sky_iterate_graph)
    hipGraphExec_t full = nullptr;
  } graphs;
  int64_t iter_count = 0;     // iterations run on this context
  int64_t switched_at = -1;   // iteration after which the ladder switched to FP64
  // phase timing: HIP event pairs on the context stream
  struct Mark { int phase, q; hipEvent_t a, b; };
  bool timing = false;
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  double ms[SKY_NPHASE][2] = {};
  int64_t cnt[SKY_NPHASE][2] = {};

  template <typename P = char> P* at(size_t off) const { return reinterpret_cast<P*>(ws + off); }
  // state buffers of set s in the current precision (phi, h phi: shared by
  // the twists of a species)
  char* psi(int s) const { return at(prec ? lay.psi32[s] : lay.psi[s]); }
  char* hpsi(int s) const { return at(prec ? lay.hpsi32[s] : lay.hpsi[s]); }
  char* phi(int s) const { return at(prec ? lay.phi32[s & 1] : lay.phi[s & 1]); }
  char* hphi(int s) const { return at(prec ? lay.hphi32[s & 1] : lay.hphi[s & 1]); }
  int m_of(int s) const { return nq[s & 1]; }
  // mean field of the species of set s (shared by every twist)
  MeanFieldPtrs mfp(int s) const {
    const double* m = at<double>(lay.mf[s & 1]);
    const float* f = at<float>(lay.mf32[s & 1]);
    return MeanFieldPtrs{m, m + n3, m + 2 * n3, f, f + n3, f + 2 * n3};
  }
  // grid arguments of set s: the Bloch shift theta / L of its twist
  GridArgs gset(int s) const {
    GridArgs r = g;
    const double L = n * d.dx;
    for (int m = 0; m < 3; ++m) r.tw[m] = d.twist[s >> 1][m] / L;
    return r;
  }
  double hb2m(int s) const { return (s & 1) ? d.hb2m_p : d.hb2m_n; }
};

namespace {
// waves per tile of the mixed plane products: 0 (untuned) selects 8
int waves_of(int w) { return w == 4 ? 4 : 8; }

hipEvent_t take_event(sky_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

// Start a timed phase; returns the mark index or -1 when timing is off.
int t_begin(sky_ctx* c, int phase, int q) {
  if (!c->timing) return -1;
  sky_ctx::Mark m{phase, q, take_event(c), take_event(c)};
  hipEventRecord(m.a, c->st);
  c->marks.push_back(m);
  return int(c->marks.size()) - 1;
}

void t_end(sky_ctx* c, int idx) {
  if (idx >= 0) hipEventRecord(c->marks[idx].b, c->st);
}

// After the stream has been synchronised: accumulate and recycle events.
void t_flush(sky_ctx* c) {
  for (auto& m : c->marks) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, m.a, m.b) == hipSuccess) {
      c->ms[m.phase][m.q] += t;
      c->cnt[m.phase][m.q] += 1;
    }
    c->pool.push_back(m.a);
    c->pool.push_back(m.b);
  }
  c->marks.clear();
}

int check_info(sky_ctx* c, const char* what) {
  int info = 0;
  int rc = hip_check(hipMemcpyAsync(&info, c->at<int>(c->lay.info), sizeof(int),
                                    hipMemcpyDeviceToHost, c->st), "info copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(c->st), what);
  if (rc) return rc;
  if (info) return fail(SKY_ERR_NOT_POSITIVE_DEFINITE, std::string(what) + ": overlap not positive definite");
  return SKY_OK;
}

// Step 3a of species q: I and H (lower triangles by the GEMMs, then
// mirrored).  Launches only, so that it can be captured in a graph.
void subspace_matrices(sky_ctx* c, int s, const void* phi, const void* hphi,
                       bool scales_ready = false) {
  const int q = s & 1;
  const int m = c->nq[q];
  hipStream_t st = c->st;
  void* I = c->at(c->lay.matI);
  void* H = c->at(c->lay.matH);
  unsigned int* mx = c->at<unsigned int>(c->lay.plS);
  if (c->prec) {
    const int tp = t_begin(c, SKY_PHASE_SPLIT, q);
    const size_t ne = size_t(m) * c->V;
    if (!scales_ready) {   // else the producers of phi and h phi merged them
      plane_scale(phi, 0, ne, mx, st);
      plane_scale(hphi, 0, ne, mx + 1, st);
    }
    split_planes_both(phi, m, c->V, mx, c->at(c->lay.plA), c->at(c->lay.plT), st);
    split_planes_nt(hphi, m, c->V, mx + 1, c->at(c->lay.plB), st);
    t_end(c, tp);
  }
  int tm = -1;
  hipEvent_t ev[2];
  if (c->timing) {
    tm = t_begin(c, SKY_PHASE_OVERLAP_GEMM, q);   // events re-recorded around the kernel
    ev[0] = c->marks[tm].a;
    ev[1] = c->marks[tm].b;
  }
  if (c->prec)
    overlap_lower_planes(c->at(c->lay.plA), c->at(c->lay.plA), c->at(c->lay.plB), mx, mx, mx + 1,
                         m, c->V, c->g.dV, I, H, c->at(c->lay.gemm_part), st,
                         c->timing ? ev : nullptr, c->tune.ovl[q], waves_of(c->tune.ovw[q]));
  else
    overlap_lower(phi, phi, hphi, m, c->V, c->g.dV, I, H, c->at(c->lay.gemm_part), st,
                  c->timing ? ev : nullptr, c->tune.ovl[q]);
  hermitian_fill(I, m, st);
  hermitian_fill(H, m, st);
}

// Steps 3b-3d of set s on the host-driven path: an orthonormalising
// transform C (C^H I C = 1), H' = C^H H C = Z lam Z^H, U = C Z.  Near the
// identity (every iteration after the start) C is Loewdin's I^-1/2 from its
// binomial series; otherwise C = L^-H with the Cholesky factor I = L L^H.
// With the paper-literal update Z and C come from H and I separately and
// U = Z C (paper_solve).
int paper_solve(sky_ctx* c, int s, double* ritz);

int jacobi_checked(sky_ctx* c, void* A, int m, double* w, void* Z) {
  const int its = jacobi_eigh(A, m, w, Z, c->at(c->lay.jac_work), JACOBI_TOL, JACOBI_SWEEPS, c->st);
  if (its == -2) return fail(SKY_ERR_NAN, "non-finite subspace matrix");
  if (its < 0) {
    ++c->unconverged;
    return JACOBI_SWEEPS;
  }
  return its;
}

int subspace_solve(sky_ctx* c, int s, double* ritz) {
  if (c->d.update == SKY_UPDATE_PAPER) return paper_solve(c, s, ritz);
  const int q = s & 1;
  const int m = c->nq[q];
  hipStream_t st = c->st;
  void* I = c->at(c->lay.matI);
  void* H = c->at(c->lay.matH);
  void* Linv = c->at(c->lay.matL);
  void* T = c->at(c->lay.matT);
  void* Hp = c->at(c->lay.matHp);
  void* Z = c->at(c->lay.matZ);
  void* U = c->at(c->lay.matU);
  int* info = c->at<int>(c->lay.info);
  const int ts = t_begin(c, SKY_PHASE_SUBSPACE, q);
  hipMemsetAsync(info, 0, sizeof(int), st);
  void* Cw = c->at(c->lay.matC);
  void* sq = c->at(c->lay.sq_part);
  const int sqs = c->tune.sq[q];
  const int terms = loewdin_series(I, Linv, Cw, T, m, LOEWDIN_SERIES_MAX,
                                   c->at<double>(c->lay.nrm), sq, st, sqs,
                                   c->prec ? MIXED_SERIES_EPS : SERIES_EPS);
  if (terms < 0) return fail(SKY_ERR_NAN, "non-finite overlap matrix");
  if (terms > 0) {   // C = I^-1/2 (Hermitian) in Linv
    gemm_square(Linv, 0, H, 0, T, m, st, sq, 0, sqs);
    gemm_square(T, 0, Linv, 0, Hp, m, st, sq, 1, sqs);
  } else {           // Linv = L^-1, C = L^-H
    hipMemcpyAsync(Cw, I, size_t(m) * m * 16, hipMemcpyDeviceToDevice, st);
    cholesky_inverse(Cw, Linv, m, c->at(c->lay.chol_work), info, st, CHOL_PIVOT_MIN);
    gemm_square(Linv, 0, H, 0, T, m, st, sq, 0, sqs);
    gemm_square(T, 0, Linv, 1, Hp, m, st, sq, 1, sqs);
  }
  hermitian_fill(Hp, m, st);   // exact Hermitian symmetry of H' before the eigensolver
  if (terms <= 0) {   // only the Cholesky path can report a non-positive overlap
    int rc = check_info(c, "cholesky");
    if (rc) return rc;
  }
  double* w = ritz ? ritz : c->at<double>(c->lay.ritz[s]);
  int its = refine_eigh(Hp, m, w, Z, c->at(c->lay.ref_work), c->prec ? REFINE_MIXED : REFINE_FP64,
                        REFINE_ITERS, st, sqs);
  if (its < 0) {   // a wide cluster or no convergence: blocked Jacobi from H'
    ++c->fallbacks;
    its = jacobi_checked(c, Hp, m, w, Z);
    if (its < 0) return its;
  }
  c->last_sweeps += its;
  gemm_square(Linv, terms > 0 ? 0 : 1, Z, 0, U, m, st, sq, 0, sqs);
  t_end(c, ts);
  return SKY_OK;
}

// Steps 3b-3d of set s with every decision on the device (launches only,
// for the captured iteration): the Loewdin series with its term count from
// the device, H', the device-decided refinement, U.  Where the host path
// would take another branch (Cholesky far from orthonormality, the Jacobi
// fallback) the box's flags hand the set to the host and mask the rest of
// the iteration.
void subspace_solve_dev(sky_ctx* c, int s) {
  const int q = s & 1;
  const int m = c->nq[q];
  hipStream_t st = c->st;
  int* fl = c->at<int>(c->lay.gflags);
  double* db = c->at<double>(c->lay.gdbl);
  void* I = c->at(c->lay.matI);
  void* H = c->at(c->lay.matH);
  void* Linv = c->at(c->lay.matL);
  void* T = c->at(c->lay.matT);
  void* Hp = c->at(c->lay.matHp);
  void* Z = c->at(c->lay.matZ);
  void* U = c->at(c->lay.matU);
  void* sq = c->at(c->lay.sq_part);
  const int sqs = c->tune.sq[q];
  loewdin_series_dev(I, Linv, c->at(c->lay.matC), T, m, LOEWDIN_SERIES_MAX,
                     c->prec ? MIXED_SERIES_EPS : SERIES_EPS, c->at<double>(c->lay.nrm), sq, st, sqs,
                     fl, db, s);
  {
    GateScope g(fl + F_ACTIVE);
    gemm_square(Linv, 0, H, 0, T, m, st, sq, 0, sqs);
    gemm_square(T, 0, Linv, 0, Hp, m, st, sq, 1, sqs);
    hermitian_fill(Hp, m, st);
  }
  refine_eigh_dev(Hp, m, c->at<double>(c->lay.ritz[s]), Z, c->at(c->lay.ref_work),
                  c->prec ? REFINE_MIXED : REFINE_FP64,
                  c->d.dev_refine_steps > 0 ? c->d.dev_refine_steps : REFINE_ITERS_DEV, st, sqs, fl, s);
  GateScope g(fl + F_ACTIVE);
  gemm_square(Linv, 0, Z, 0, U, m, st, sq, 0, sqs);
}

// Unitary polar factor P of the k x k complex matrix G (row-major; G = P S
// with S Hermitian positive semi-definite) by Newton's iteration
// X <- (X + X^-H) / 2 from X = G (quadratic convergence for a non-singular
// G).  Returns false when G is numerically singular or the iteration does
// not settle.
bool polar_unitary(const std::vector<std::complex<double>>& G, int k,
                   std::vector<std::complex<double>>& P) {
  using cd = std::complex<double>;
  P = G;
  std::vector<cd> A(size_t(k) * 2 * k);
  for (int it = 0; it < 60; ++it) {
    // inverse of X by Gauss-Jordan with partial pivoting on [X | 1]
    for (int r = 0; r < k; ++r)
      for (int col = 0; col < 2 * k; ++col)
        A[size_t(r) * 2 * k + col] = col < k ? P[size_t(r) * k + col] : cd(col - k == r ? 1.0 : 0.0);
    double scale = 0.0;
    for (int e = 0; e < k * k; ++e) scale = std::max(scale, std::abs(P[e]));
    for (int col = 0; col < k; ++col) {
      int piv = col;
      for (int r = col + 1; r < k; ++r)
        if (std::abs(A[size_t(r) * 2 * k + col]) > std::abs(A[size_t(piv) * 2 * k + col])) piv = r;
      if (!(std::abs(A[size_t(piv) * 2 * k + col]) > 1e-10 * scale)) return false;
      if (piv != col)
        for (int e = 0; e < 2 * k; ++e) std::swap(A[size_t(piv) * 2 * k + e], A[size_t(col) * 2 * k + e]);
      const cd inv = 1.0 / A[size_t(col) * 2 * k + col];
      for (int e = 0; e < 2 * k; ++e) A[size_t(col) * 2 * k + e] *= inv;
      for (int r = 0; r < k; ++r) {
        if (r == col) continue;
        const cd f = A[size_t(r) * 2 * k + col];
        if (f == cd(0.0)) continue;
        for (int e = 0; e < 2 * k; ++e) A[size_t(r) * 2 * k + e] -= f * A[size_t(col) * 2 * k + e];
      }
    }
    // X <- (X + X^-H) / 2
    double change = 0.0;
    for (int r = 0; r < k; ++r)
      for (int col = 0; col < k; ++col) {
        const cd xinvh = std::conj(A[size_t(col) * 2 * k + k + r]);
        const cd nx = 0.5 * (P[size_t(r) * k + col] + xinvh);
        change = std::max(change, std::abs(nx - P[size_t(r) * k + col]));
        P[size_t(r) * k + col] = nx;
      }
    if (change < 1e-15) return true;
  }
  return false;
}

// The paper-literal update of Sec. 3.3.3 for set s: Z from the Hermitian
// eigenproblem of H alone (3b), C = I^-1/2 from I alone (3c), U = Z C (3d).
// Z is brought to the gauge closest to the identity: within each cluster of
// eigenvalues closer than PAPER_CLUSTER_TOL the columns are rotated by
// Q = P^H, P the unitary polar factor of the cluster's diagonal block (a
// single state: the phase that makes Z_bb real and positive).
int paper_solve(sky_ctx* c, int s, double* ritz) {
  const int q = s & 1;
  const int m = c->nq[q];
  hipStream_t st = c->st;
  void* I = c->at(c->lay.matI);
  void* H = c->at(c->lay.matH);
  void* C = c->at(c->lay.matL);
  void* T = c->at(c->lay.matT);
  void* X = c->at(c->lay.matHp);
  void* Z = c->at(c->lay.matZ);
  void* U = c->at(c->lay.matU);
  void* Cw = c->at(c->lay.matC);
  void* sq = c->at(c->lay.sq_part);
  int* info = c->at<int>(c->lay.info);
  const int sqs = c->tune.sq[q];
  const int ts = t_begin(c, SKY_PHASE_SUBSPACE, q);
  hipMemsetAsync(info, 0, sizeof(int), st);
  // 3c: C = I^-1/2, by the series near the identity, else by the eigenvectors of I
  const int terms = loewdin_series(I, C, Cw, T, m, LOEWDIN_SERIES_MAX,
                                   c->at<double>(c->lay.nrm), sq, st, sqs);
  if (terms < 0) return fail(SKY_ERR_NAN, "non-finite overlap matrix");
  if (terms == 0) {
    double* wi = c->at<double>(c->lay.wtmp);
    hipMemcpyAsync(Cw, I, size_t(m) * m * 16, hipMemcpyDeviceToDevice, st);
    int rc = jacobi_checked(c, Cw, m, wi, X);
    if (rc < 0) return rc;
    hipMemcpyAsync(T, X, size_t(m) * m * 16, hipMemcpyDeviceToDevice, st);
    inv_sqrt(wi, m, info, st, CHOL_PIVOT_MIN);
    scale_columns(T, wi, m, st);
    gemm_square(T, 0, X, 1, C, m, st, sq, 1, sqs);
    rc = check_info(c, "paper update: overlap");
    if (rc) return rc;
  }
  // 3b: H Z = Z lam (ascending)
  double* w = ritz ? ritz : c->at<double>(c->lay.ritz[s]);
  const RefineTargets tg{JACOBI_TOL, c->prec ? MIXED_HP_NOISE : 0x1p-49, REFINE_FP64.orth,
                         REFINE_FP64.e2skip};
  int its = refine_eigh(H, m, w, Z, c->at(c->lay.ref_work), tg, REFINE_ITERS, st, sqs);
  if (its < 0) {
    ++c->fallbacks;
    hipMemcpyAsync(X, H, size_t(m) * m * 16, hipMemcpyDeviceToDevice, st);
    its = jacobi_checked(c, X, m, w, Z);
    if (its < 0) return its;
  }
  c->last_sweeps += its;
  // gauge of Z: clusters from the eigenvalues, diagonal blocks to the host
  std::vector<double> lam(m);
  int rc = hip_check(hipMemcpyAsync(lam.data(), w, sizeof(double) * m, hipMemcpyDeviceToHost, st),
                     "eigenvalue copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(st), "paper update");
  if (rc) return rc;
  std::vector<int> info3(size_t(3) * m);   // per column: cluster start, size, block offset
  size_t packed = 0;
  for (int a = 0; a < m;) {
    int b = a + 1;
    while (b < m && lam[b] - lam[b - 1] < PAPER_CLUSTER_TOL) ++b;
    for (int col = a; col < b; ++col) {
      info3[3 * col] = a;
      info3[3 * col + 1] = b - a;
      info3[3 * col + 2] = int(packed);
    }
    packed += size_t(b - a) * (b - a);
    a = b;
  }
  int* dinfo = c->at<int>(c->lay.gauge);
  hipMemcpyAsync(dinfo, info3.data(), sizeof(int) * info3.size(), hipMemcpyHostToDevice, st);
  gauge_gather(Z, m, dinfo, T, st);
  std::vector<std::complex<double>> blocks(packed);
  rc = hip_check(hipMemcpyAsync(blocks.data(), T, packed * 16, hipMemcpyDeviceToHost, st),
                 "gauge block copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(st), "paper update");
  if (rc) return rc;
  std::vector<std::complex<double>> G, P;
  for (int a = 0; a < m;) {
    const int k = info3[3 * a + 1];
    const size_t off = size_t(info3[3 * a + 2]);
    G.assign(blocks.begin() + off, blocks.begin() + off + size_t(k) * k);
    if (polar_unitary(G, k, P)) {
      for (int r = 0; r < k; ++r)   // Q = P^H
        for (int col = 0; col < k; ++col) blocks[off + size_t(r) * k + col] = std::conj(P[size_t(col) * k + r]);
    } else {                        // singular block: phases only
      for (int r = 0; r < k; ++r)
        for (int col = 0; col < k; ++col) {
          const std::complex<double> z = G[size_t(col) * k + col];
          blocks[off + size_t(r) * k + col] =
              r == col ? (std::abs(z) > 0.0 ? std::conj(z) / std::abs(z) : 1.0) : 0.0;
        }
    }
    a += k;
  }
  hipMemcpyAsync(T, blocks.data(), packed * 16, hipMemcpyHostToDevice, st);
  gauge_apply(Z, m, dinfo, T, X, st);     // X = Z Q (block-diagonal Q)
  // 3d: U = Z C
  gemm_square(X, 0, C, 0, U, m, st, sq, 0, sqs);
  rc = hip_check(hipStreamSynchronize(st), "paper update");   // host blocks leave scope
  if (rc) return rc;
  t_end(c, ts);
  return SKY_OK;
}

// Step 3e of set s: psi = phi U (launches only).  With one_h the h phi of
// the update is carried along: h psi = (h phi) U.
void subspace_combine(sky_ctx* c, int s, const void* phi, void* psi_out,
                      const void* hphi = nullptr, void* hpsi_out = nullptr) {
  const int q = s & 1;
  const int m = c->nq[q];
  hipStream_t st = c->st;
  void* U = c->at(c->lay.matU);
  unsigned int* mx = c->at<unsigned int>(c->lay.plS);
  const int tc = t_begin(c, SKY_PHASE_COMBINE_GEMM, q);
  if (c->prec) {
    plane_scale(U, 1, size_t(m) * m, mx + 2, st);
    split_planes_t(U, 1, m, m, mx + 2, c->at(c->lay.plU), st);
    combine_planes(c->at(c->lay.plU), c->at(c->lay.plT), mx + 2, mx, psi_out, m, c->V, st,
                   waves_of(c->tune.cbw[q]));
    if (hphi) {   // the planes of (h phi)^T replace those of phi^T
      split_planes_t(hphi, 0, m, c->V, mx + 1, c->at(c->lay.plT), st);
      combine_planes(c->at(c->lay.plU), c->at(c->lay.plT), mx + 2, mx + 1, hpsi_out, m, c->V, st,
                     waves_of(c->tune.cbw[q]));
    }
  } else {
    combine(phi, U, psi_out, m, c->V, st);
    if (hphi) combine(hphi, U, hpsi_out, m, c->V, st);
  }
  t_end(c, tc);
}

// Generalised Rayleigh-Ritz on phi/hphi of set s -> psi_out (Sec. 3.3).
int rayleigh_ritz(sky_ctx* c, int s, const void* phi, const void* hphi, void* psi_out,
                  double* ritz) {
  if (c->m_of(s) == 0) return SKY_OK;
  subspace_matrices(c, s, phi, hphi);
  int rc = subspace_solve(c, s, ritz);
  if (rc) return rc;
  subspace_combine(c, s, phi, psi_out);
  return SKY_OK;
}

int loewdin(sky_ctx* c, int s, const void* phi, void* psi_out) {
  const int q = s & 1;
  const int m = c->nq[q];
  if (m == 0) return SKY_OK;
  hipStream_t st = c->st;
  void* I = c->at(c->lay.matI);
  void* X = c->at(c->lay.matZ);
  void* C = c->at(c->lay.matU);
  double* w = c->at<double>(c->lay.ritz[s]);
  int* info = c->at<int>(c->lay.info);
  hipMemsetAsync(info, 0, sizeof(int), st);
  unsigned int* mx = c->at<unsigned int>(c->lay.plS);
  if (c->prec) {
    plane_scale(phi, 0, size_t(m) * c->V, mx, st);
    split_planes_both(phi, m, c->V, mx, c->at(c->lay.plA), c->at(c->lay.plT), st);
    overlap_lower_planes(c->at(c->lay.plA), c->at(c->lay.plA), nullptr, mx, mx, nullptr, m,
                         c->V, c->g.dV, I, nullptr, c->at(c->lay.gemm_part), st, nullptr,
                         c->tune.ovl[q]);
  } else
    overlap_lower(phi, phi, nullptr, m, c->V, c->g.dV, I, nullptr, c->at(c->lay.gemm_part), st,
                  nullptr, c->tune.ovl[q]);
  hermitian_fill(I, m, st);
  int its = jacobi_checked(c, I, m, w, X);
  if (its < 0) return its;
  // C = X diag(w^-1/2) X^H
  double* wi = c->at<double>(c->lay.wtmp);
  hipMemcpyAsync(c->at(c->lay.matT), X, size_t(m) * m * 16, hipMemcpyDeviceToDevice, st);
  hipMemcpyAsync(wi, w, sizeof(double) * m, hipMemcpyDeviceToDevice, st);
  inv_sqrt(wi, m, info, st, CHOL_PIVOT_MIN);
  scale_columns(c->at(c->lay.matT), wi, m, st);
  gemm_square(c->at(c->lay.matT), 0, X, 1, C, m, st, c->at(c->lay.sq_part), 1, c->tune.sq[q]);
  int rc = check_info(c, "loewdin");
  if (rc) return rc;
  if (c->prec) {
    plane_scale(C, 1, size_t(m) * m, mx + 2, st);
    split_planes_t(C, 1, m, m, mx + 2, c->at(c->lay.plU), st);
    combine_planes(c->at(c->lay.plU), c->at(c->lay.plT), mx + 2, mx, psi_out, m, c->V, st);
  } else {
    combine(phi, C, psi_out, m, c->V, st);
  }
  return SKY_OK;
}

// Fig. 1 steps 4a, 4b, 5: densities of the occupied states of every set,
// averaged over the twists, then mean field, Coulomb and energy.
void fields(sky_ctx* c) {
  hipStream_t st = c->st;
  const void* ps[SKY_MAX_TWIST];
  GridArgs gs[SKY_MAX_TWIST];
  for (int q = 0; q < 2; ++q) {
    const int td = t_begin(c, SKY_PHASE_DENSITIES, q);
    for (int t = 0; t < c->ntw; ++t) {
      ps[t] = c->psi(2 * t + q);
      gs[t] = c->gset(2 * t + q);
    }
    (void)sky::densities(c->n, c->prec, ps, gs, c->ntw, c->nocc[q], DENS_CHUNKS,
                   c->at<double>(c->lay.dens_part), c->at<double>(c->lay.dens[q]), st);
    t_end(c, td);
  }
  const int tmf = t_begin(c, SKY_PHASE_MEANFIELD, 0);
  mean_field(c->n, c->g, c->sk, c->at<double>(c->lay.dens[0]), c->at<double>(c->lay.dens[1]),
             c->at<double>(c->lay.der[0]), c->at<double>(c->lay.der[1]),
             c->at<double>(c->lay.mf[0]), c->at<double>(c->lay.mf[1]),
             c->at<double>(c->lay.vc), c->at(c->lay.fscratch), c->at<double>(c->lay.epart),
             c->at<double>(c->lay.energy), st);
  // FP32 copies of U, B, W for the complex64 kernels (5 n^3 doubles as
  // complex pairs: n^3 is even)
  for (int q = 0; q < 2; ++q)
    convert_states(c->at(c->lay.mf[q]), 0, c->at(c->lay.mf32[q]), 1, size_t(5) * c->n3 / 2, st);
  t_end(c, tmf);
}
// |k| at the corner of the Brillouin zone
double kmax_of(const sky_ctx* c) { return std::sqrt(3.0) * (c->n / 2) * c->g.kunit; }

// Damped step with the learned per-shell gains: forward passes and shell
// powers, MLP inference of the gains, then the gained filter and inverses.
void learned_damp(sky_ctx* c, int s, const void* psi, const void* hpsi, const double* eps,
                  void* phi, int m, double* r2, hipStream_t st, unsigned int* amax = nullptr) {
  const double hb = c->hb2m(s);
  const GridArgs gs = c->gset(s);
  double* pw = c->at<double>(c->lay.pc_pow);
  zero(pw, size_t(m) * PC_SHELLS, st);
  damped_step(c->n, c->prec, psi, hpsi, eps, phi, m, gs, c->d.damp_x0, c->d.damp_e0, hb,
              c->at<double>(c->lay.tiles), r2, st, nullptr, pw, 1, c->tune.damp_xy);
  float* X = c->at<float>(c->lay.pc_X);
  precond_features(pw, eps, 1, m, c->d.damp_e0, hb, kmax_of(c), X, st);
  precond_forward(c->at<float>(c->lay.pc_Pb), X, m * PC_SHELLS, nullptr, nullptr, nullptr,
                  c->at<float>(c->lay.pc_O), st);
  precond_gains(c->at<float>(c->lay.pc_O), m * PC_SHELLS, c->at<float>(c->lay.pc_gain), st);
  damped_step(c->n, c->prec, psi, hpsi, eps, phi, m, gs, c->d.damp_x0, c->d.damp_e0, hb,
              nullptr, nullptr, st, c->at<float>(c->lay.pc_gain), nullptr, 2, c->tune.damp_xy,
              amax);
}

// Training rows from the current states of set s: the shell powers and
// features of up to NS_MAX evenly spaced states, their one-shell damped
// directions d_s, h d_s and the target gains.  Rows go to a ring of PC_CAP
// rows (a collection that does not fit at the end starts again at row 0).
int pc_collect(sky_ctx* c, int s) {
  hipStream_t st = c->st;
  const int m = c->m_of(s);
  const GridArgs gs = c->gset(s);
  const int ns = std::min(precond_ns_max(), m);
  if (ns <= 0) return SKY_OK;
  const int nb = ns * PC_SHELLS;
  if (c->pc_wr + nb > PC_CAP) c->pc_wr = 0;
  std::vector<int> idx(ns);
  for (int a = 0; a < ns; ++a) idx[a] = int((long(a) * m) / ns);
  int* didx = c->at<int>(c->lay.pc_idx);
  hipMemcpyAsync(didx, idx.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st);
  double* eps = c->at<double>(c->lay.eps[s]);
  double* tiles = c->at<double>(c->lay.tiles);
  c->hpsi_lagged = false;   // h psi is rebuilt with the current mean field here
  apply_h(c->n, c->prec, c->psi(s), c->hpsi(s), m, c->mfp(s), gs, tiles, eps, st,
          c->tune.lines);
  void* b0 = c->at(c->lay.pc_b[0]);   // psi copies
  void* b1 = c->at(c->lay.pc_b[1]);   // h psi copies
  void* b2 = c->at(c->lay.pc_b[2]);   // phi, then the shell directions d
  void* b3 = c->at(c->lay.pc_b[3]);   // h d
  double* beps = c->at<double>(c->lay.pc_beps);
  float* onehot = c->at<float>(c->lay.pc_gain);
  double* pw = c->at<double>(c->lay.pc_pow);
  precond_gather(c->prec, c->psi(s), c->hpsi(s), eps, didx, ns, c->V, b0, b1, beps, onehot, st);
  zero(pw, size_t(nb) * PC_SHELLS, st);
  const double hb = c->hb2m(s);
  damped_step(c->n, c->prec, b0, b1, beps, b2, nb, gs, c->d.damp_x0, c->d.damp_e0, hb, tiles,
              nullptr, st, onehot, pw, 0, c->tune.damp_xy);
  float* rows = c->at<float>(c->lay.pc_S) + size_t(c->pc_wr) * 6;
  precond_features(pw, beps, PC_SHELLS, ns, c->d.damp_e0, hb, kmax_of(c), rows, st);
  precond_dir(c->prec, b0, b2, size_t(nb) * c->V, st);
  apply_h(c->n, c->prec, b2, b3, nb, c->mfp(s), gs, nullptr, nullptr, st, c->tune.lines);
  precond_targets(c->prec, b0, b1, b2, b3, beps, ns, c->V, c->at<double>(c->lay.pc_gram), rows,
                  st);
  int rc = hip_check(hipStreamSynchronize(st), "precond_collect");
  if (rc) return rc;
  c->pc_wr += nb;
  c->pc_count = std::max(c->pc_count, c->pc_wr);
  return SKY_OK;
}

double precond_wsum(sky_ctx* c) {
  std::vector<float> rows(size_t(c->pc_count) * 6);
  hipMemcpyAsync(rows.data(), c->at(c->lay.pc_S), sizeof(float) * rows.size(),
                 hipMemcpyDeviceToHost, c->st);
  hipStreamSynchronize(c->st);
  double w = 0.0;
  for (int b = 0; b < c->pc_count; ++b) w += rows[size_t(b) * 6 + 5];
  return w > 0.0 ? w : 1.0;
}

double precond_pass(sky_ctx* c, double wsum, int want_loss) {
  return precond_loss_grad(
      c->at<float>(c->lay.pc_Pb), c->at<float>(c->lay.pc_S), c->pc_count, wsum,
      c->at<float>(c->lay.pc_H[0]), c->at<float>(c->lay.pc_H[1]), c->at<float>(c->lay.pc_H[2]),
      c->at<float>(c->lay.pc_O), c->at<float>(c->lay.pc_dO), c->at<float>(c->lay.pc_D[0]),
      c->at<float>(c->lay.pc_D[1]), c->at<float>(c->lay.pc_D[2]), c->at<float>(c->lay.pc_G),
      c->at<float>(c->lay.pc_gpart), c->at<double>(c->lay.pc_dscr), want_loss, c->st);
}

// Adam over every held row; returns the loss before the last update.
double pc_train(sky_ctx* c, int steps, double lr) {
  const double w = precond_wsum(c);
  double l = 0.0;
  for (int s = 1; s <= steps; ++s) {
    precond_round(c->at<float>(c->lay.pc_P), c->at<float>(c->lay.pc_Pb), c->st);
    l = precond_pass(c, w, s == steps);
    precond_adam(c->at<float>(c->lay.pc_P), c->at<float>(c->lay.pc_G), c->at<float>(c->lay.pc_M),
                 c->at<float>(c->lay.pc_V), ++c->pc_step, float(lr), c->st);
  }
  precond_round(c->at<float>(c->lay.pc_P), c->at<float>(c->lay.pc_Pb), c->st);
  c->pc_trained = true;
  c->pc_lr = lr;
  return l;
}

// Step 2 and step 3a of set s: h psi and <h> (or, with one_h after an
// update, the h psi carried over and <h> = the subspace eigenvalues), the
// damped step (plain or learned), h phi, then I and H.  Launches only.
void step_a(sky_ctx* c, int s, bool learned, bool lagged) {
  const int q = s & 1;
  const int m = c->nq[q];
  hipStream_t st = c->st;
  void* psi = c->psi(s);
  void* hpsi = c->hpsi(s);
  void* phi = c->phi(s);
  void* hphi = c->hphi(s);
  const GridArgs gs = c->gset(s);
  double* eps = c->at<double>(c->lay.eps[s]);
  double* tiles = c->at<double>(c->lay.tiles);
  // mixed: the largest |component| of phi and h phi (split-plane scales) is
  // merged by the kernels that write them
  unsigned int* mx = c->prec ? c->at<unsigned int>(c->lay.plS) : nullptr;
  if (mx) clear_scales(mx, 2, st);
  if (lagged) {
    hipMemcpyAsync(eps, c->at(c->lay.ritz[s]), sizeof(double) * m, hipMemcpyDeviceToDevice, st);
  } else {
    int t0 = t_begin(c, SKY_PHASE_APPLY_H, q);
    apply_h(c->n, c->prec, psi, hpsi, m, c->mfp(s), gs, tiles, eps, st, c->tune.lines);
    t_end(c, t0);
  }
  const double hb = c->hb2m(s);
  int t1 = t_begin(c, SKY_PHASE_DAMP, q);
  if (learned)
    learned_damp(c, s, psi, hpsi, eps, phi, m, c->at<double>(c->lay.r2[s]), st, mx);
  else
    damped_step(c->n, c->prec, psi, hpsi, eps, phi, m, gs, c->d.damp_x0, c->d.damp_e0, hb,
                tiles, c->at<double>(c->lay.r2[s]), st, nullptr, nullptr, 0, c->tune.damp_xy, mx);
  t_end(c, t1);
  int t2 = t_begin(c, SKY_PHASE_APPLY_H, q);
  apply_h(c->n, c->prec, phi, hphi, m, c->mfp(s), gs, nullptr, nullptr, st, c->tune.lines,
          mx ? mx + 1 : nullptr);
  t_end(c, t2);
  subspace_matrices(c, s, phi, hphi, mx != nullptr);
}

void graphs_clear(sky_ctx* c) {
  auto drop = [](hipGraphExec_t& g) { if (g) { hipGraphExecDestroy(g); g = nullptr; } };
  for (int s = 0; s < MAXSET; ++s) {
    for (int v = 0; v < 4; ++v) drop(c->graphs.a[s][v]);
    drop(c->graphs.b[s]);
  }
  drop(c->graphs.f);
  drop(c->graphs.full);
}

// Runs body's launches: directly, or (graphs on, timing off) by replaying the
// graph captured from body at its first use.  Graphs hold the context's
// buffers, sizes, precision and launch shapes; they are dropped whenever one
// of those changes.
template <class Body>
int run_segment(sky_ctx* c, hipGraphExec_t& exec, Body&& body) {
  if (!c->graphs.on || c->timing) {
    body();
    return SKY_OK;
  }
  if (c->graphs.prec != c->prec) {
    hipStreamSynchronize(c->st);
    graphs_clear(c);
    c->graphs.prec = c->prec;
  }
  if (!exec) {
    hipGraph_t g = nullptr;
    int rc = hip_check(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal), "graph capture");
    if (rc) return rc;
    body();
    rc = hip_check(hipStreamEndCapture(c->st, &g), "graph capture");
    if (rc) return rc;
    rc = hip_check(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0), "graph instantiate");
    hipGraphDestroy(g);
    if (rc) return rc;
    ++c->graphs.captures;
  }
  return hip_check(hipGraphLaunch(exec, c->st), "graph launch");
}

// ------------------------------------------------------------------ autotuning
// Flat JSON cache {"key": integer, ...}; keys name the operation, its sizes
// and the precision.  Unreadable or absent files count as empty.
std::vector<std::pair<std::string, int>> cache_read(const char* path) {
  std::vector<std::pair<std::string, int>> kv;
  if (!path) return kv;
  FILE* f = std::fopen(path, "r");
  if (!f) return kv;
  std::string txt;
  char buf[4096];
  size_t nread;
  while ((nread = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, nread);
  std::fclose(f);
  size_t i = 0;
  while ((i = txt.find('"', i)) != std::string::npos) {
    const size_t j = txt.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = txt.substr(i + 1, j - i - 1);
    size_t k = txt.find(':', j);
    if (k == std::string::npos) break;
    ++k;
    while (k < txt.size() && (txt[k] == ' ' || txt[k] == '\t' || txt[k] == '\n')) ++k;
    char* end = nullptr;
    const long v = std::strtol(txt.c_str() + k, &end, 10);
    if (end != txt.c_str() + k) kv.emplace_back(key, int(v));
    i = end ? size_t(end - txt.c_str()) : j + 1;
  }
  return kv;
}

bool cache_write(const char* path, const std::vector<std::pair<std::string, int>>& kv) {
  if (!path) return true;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < kv.size(); ++i)
    std::fprintf(f, "  \"%s\": %d%s\n", kv[i].first.c_str(), kv[i].second, i + 1 < kv.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
  return std::rename(tmp.c_str(), path) == 0;
}

int cache_get(const std::vector<std::pair<std::string, int>>& kv, const std::string& key) {
  for (const auto& e : kv)
    if (e.first == key) return e.second;
  return 0;
}

bool cache_has(const std::vector<std::pair<std::string, int>>& kv, const std::string& key) {
  for (const auto& e : kv)
    if (e.first == key) return true;
  return false;
}

void cache_put(std::vector<std::pair<std::string, int>>& kv, const std::string& key, int v) {
  for (auto& e : kv)
    if (e.first == key) { e.second = v; return; }
  kv.emplace_back(key, v);
}

// Mean milliseconds of `reps` runs of op (after one untimed run).
template <typename F> double time_op(hipStream_t st, int reps, F op) {
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  op();
  hipEventRecord(a, st);
  for (int r = 0; r < reps; ++r) op();
  hipEventRecord(b, st);
  hipEventSynchronize(b);
  float ms = 0.0f;
  hipEventElapsedTime(&ms, a, b);
  hipEventDestroy(a);
  hipEventDestroy(b);
  return double(ms) / reps;
}

// Fastest candidate of op(candidate).
template <typename F> int pick(hipStream_t st, const int* cand, int nc, F op) {
  int best = cand[0];
  double tb = 1e300;
  for (int i = 0; i < nc; ++i) {
    const double t = time_op(st, 3, [&] { op(cand[i]); });
    if (t < tb) { tb = t; best = cand[i]; }
  }
  return best;
}

// ------------------------------------------------------------------ device-decided iteration
// Whether the context can run the captured iteration whose decisions are
// made on the device.  Options whose decisions stay on the host (the learned
// damping's fallback rule and online training, the precision ladder, the
// paper-literal update, one h application, phase timing) and a context on
// the null stream (no capture there) run sky_iterate instead.
bool dev_iteration_ok(const sky_ctx* c) {
  return !c->timing && c->d.update == SKY_UPDATE_EXACT && !c->d.one_h && !c->pc_on &&
         !(c->prec == 1 && c->d.ladder_tol > 0.0) && c->st != nullptr;
}

// Delta-eps of the iteration, the iteration count and the convergence test,
// on the device (k_iteration_end).
void dev_iteration_end(sky_ctx* c) {
  const double* r2[MAXSET];
  int nocc[MAXSET];
  for (int s = 0; s < c->nset; ++s) {
    r2[s] = c->at<double>(c->lay.r2[s]);
    nocc[s] = c->m_of(s) ? c->nocc[s & 1] : 0;
  }
  iteration_end(r2, nocc, c->nset, c->ntw * (c->nocc[0] + c->nocc[1]), c->at<int>(c->lay.gflags),
                c->at<double>(c->lay.gdbl), c->st);
}

// One iteration (every set, the fields, Delta-eps), each kernel gated by the
// box's flags: launches only, captured once per context and precision.
void iteration_dev(sky_ctx* c) {
  int* fl = c->at<int>(c->lay.gflags);
  for (int s = 0; s < c->nset; ++s) {
    if (c->m_of(s) == 0) continue;
    {
      GateScope g(fl + F_ACTIVE);
      step_a(c, s, false, false);
    }
    subspace_solve_dev(c, s);
    GateScope g(fl + F_ACTIVE);
    subspace_combine(c, s, c->phi(s), c->psi(s));
  }
  {
    GateScope g(fl + F_ACTIVE);
    fields(c);
  }
  dev_iteration_end(c);
}

// The rest of an iteration on the host path, from the solve of set s0 (its
// phi, h phi, I and H are in place) when the device handed it over; then
// the box is active again and Delta-eps is taken on the device.
int resume_on_host(sky_ctx* c, int s0) {
  for (int s = s0; s < c->nset; ++s) {
    if (c->m_of(s) == 0) continue;
    if (s > s0) step_a(c, s, false, false);
    int rc = subspace_solve(c, s, c->at<double>(c->lay.ritz[s]));
    if (rc) return rc;
    subspace_combine(c, s, c->phi(s), c->psi(s));
  }
  fields(c);
  int* fl = c->at<int>(c->lay.gflags);
  set_flag(fl, F_HOST, HOST_NONE, c->st);
  set_flag(fl, F_ACTIVE, 1, c->st);
  dev_iteration_end(c);
  return SKY_OK;
}

int capture_full(sky_ctx* c) {
  if (c->graphs.prec != c->prec) {
    hipStreamSynchronize(c->st);
    graphs_clear(c);
    c->graphs.prec = c->prec;
  }
  if (c->graphs.full) return SKY_OK;
  hipGraph_t g = nullptr;
  int rc = hip_check(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal), "graph capture");
  if (rc) return rc;
  iteration_dev(c);
  rc = hip_check(hipStreamEndCapture(c->st, &g), "graph capture");
  if (rc) return rc;
  rc = hip_check(hipGraphInstantiate(&c->graphs.full, g, nullptr, nullptr, 0), "graph instantiate");
  hipGraphDestroy(g);
  if (rc) return rc;
  ++c->graphs.captures;
  return SKY_OK;
}

// A device-decided run of one context: started, then launched and collected
// chunk by chunk (the host reads the flags once per chunk).
struct DevRun {
  sky_ctx* c = nullptr;
  int max_iter = 0, chunk = 1;
  double tol = 0.0;
  int done = 0;        // iterations completed
  int handovers = 0;   // iterations finished on the host path
  bool finished = false;
  int status = SKY_OK;
  int flags[F_NFLAGS] = {};
  double dbl[D_NDOUBLES] = {};
};

int dev_start(DevRun& r) {
  sky_ctx* c = r.c;
  c->fallbacks = 0;
  c->unconverged = 0;
  c->pc_iters = 0;
  int* fl = c->at<int>(c->lay.gflags);
  for (int f = 0; f < F_NFLAGS; ++f) set_flag(fl, f, f == F_ACTIVE ? 1 : 0, c->st);
  set_double(c->at<double>(c->lay.gdbl), D_TOL, r.tol > 0.0 ? r.tol : 0.0, c->st);
  set_double(c->at<double>(c->lay.gdbl), D_DE, 0.0, c->st);
  if (r.max_iter == 0) r.finished = true;
  return capture_full(c);
}

int dev_launch(DevRun& r) {
  if (r.finished) return SKY_OK;
  const int k = std::min(r.chunk, r.max_iter - r.done);
  for (int i = 0; i < k; ++i) {
    int rc = hip_check(hipGraphLaunch(r.c->graphs.full, r.c->st), "graph launch");
    if (rc) return rc;
  }
  return SKY_OK;
}

int dev_read(DevRun& r) {
  sky_ctx* c = r.c;
  int rc = hip_check(hipMemcpyAsync(r.flags, c->at(c->lay.gflags), sizeof(r.flags),
                                    hipMemcpyDeviceToHost, c->st), "flags copy");
  if (rc) return rc;
  rc = hip_check(hipMemcpyAsync(r.dbl, c->at(c->lay.gdbl), sizeof(r.dbl), hipMemcpyDeviceToHost,
                                c->st), "flags copy");
  if (rc) return rc;
  return hip_check(hipStreamSynchronize(c->st), "iterate_graph");
}

// After the stream has drained: read the flags, finish a handed-over
// iteration on the host, decide whether the run is done.
int dev_collect(DevRun& r) {
  if (r.finished) return SKY_OK;
  int rc = dev_read(r);
  if (rc) return rc;
  if (r.flags[F_HOST] == HOST_NAN) return fail(SKY_ERR_NAN, "non-finite residual");
  if (r.flags[F_HOST] != HOST_NONE) {
    rc = resume_on_host(r.c, r.flags[F_HOST_SET]);
    if (rc) return rc;
    ++r.handovers;
    rc = dev_read(r);
    if (rc) return rc;
    if (r.flags[F_HOST] == HOST_NAN) return fail(SKY_ERR_NAN, "non-finite residual");
  }
  r.done = r.flags[F_ITER];
  if (r.flags[F_CONV]) {
    r.finished = true;
    r.status = SKY_OK;
  } else if (r.done >= r.max_iter) {
    r.finished = true;
    r.status = r.tol > 0.0 ? SKY_NOT_CONVERGED : SKY_OK;
  }
  return SKY_OK;
}

int dev_finish(DevRun& r, sky_report* rep) {
  sky_ctx* c = r.c;
  double e[8] = {0};
  int rc = hip_check(hipMemcpyAsync(e, c->at(c->lay.energy), sizeof(e), hipMemcpyDeviceToHost, c->st),
                     "energy copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(c->st), "iterate_graph");
  if (rc) return rc;
  if (!std::isfinite(e[7])) return fail(SKY_ERR_NAN, "non-finite energy");
  c->iter_count += r.done;
  c->de_prev = r.dbl[D_DE];
  if (rep) {
    rep->precision = c->prec ? SKY_MIXED : SKY_FP64;
    rep->iters = r.done;
    rep->residual = r.dbl[D_DE];
    rep->energy = e[7];
    rep->energy_per_a = e[7] / double(std::max(1, c->nocc[0] + c->nocc[1]));
    rep->eig_iters = r.flags[F_REF_STEPS];
    rep->eig_fallbacks = r.handovers;
    rep->precond_iters = 0;
    rep->eig_unconverged = c->unconverged;
  }
  return r.status;
}
}  // namespace


extern "C" {

int sky_workspace_size(const sky_box_desc* d, size_t* bytes) {
  int rc = validate(d);
  if (rc) return rc;
  if (!bytes) return fail(SKY_ERR_INVALID, "null bytes");
  *bytes = plan(*d).total;
  return SKY_OK;
}

int sky_create(const sky_box_desc* d, void* workspace, size_t bytes, void* stream, sky_ctx** out) {
  int rc = validate(d);
  if (rc) return rc;
  if (!out) return fail(SKY_ERR_INVALID, "null out");
  Layout L = plan(*d);
  if (!workspace || bytes < L.total) return fail(SKY_ERR_WORKSPACE, "workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % ALIGN) return fail(SKY_ERR_WORKSPACE, "workspace not 256-byte aligned");
  sky_ctx* c = new sky_ctx();
  c->d = *d;
  c->lay = L;
  c->ws = static_cast<char*>(workspace);
  c->st = static_cast<hipStream_t>(stream);
  c->n = d->n;
  c->n3 = d->n * d->n * d->n;
  c->V = 2L * c->n3;
  c->nq[0] = states_of(*d, 0);
  c->nq[1] = states_of(*d, 1);
  c->nocc[0] = d->n_neutrons;
  c->nocc[1] = d->n_protons;
  c->ntw = ntwist_of(*d);
  c->nset = 2 * c->ntw;
  c->prec = d->precision == SKY_MIXED ? 1 : 0;
  c->g.dx = d->dx;
  c->g.dV = d->dx * d->dx * d->dx;
  c->g.kunit = 2.0 * M_PI / (d->n * d->dx);
  c->g.tw[0] = c->g.tw[1] = c->g.tw[2] = 0.0;
  const double t0 = d->t0, t1 = d->t1, t2 = d->t2, t3 = d->t3;
  const double x0 = d->x0, x1 = d->x1, x2 = d->x2, x3 = d->x3;
  // b-coefficients of the Skyrme functional (standard t/x -> b mapping)
  c->sk.b0 = t0 * (1 + x0 / 2);
  c->sk.b0p = t0 * (0.5 + x0);
  c->sk.b1 = (t1 * (1 + x1 / 2) + t2 * (1 + x2 / 2)) / 4;
  c->sk.b1p = (t1 * (0.5 + x1) - t2 * (0.5 + x2)) / 4;
  c->sk.b2 = (3 * t1 * (1 + x1 / 2) - t2 * (1 + x2 / 2)) / 8;
  c->sk.b2p = (3 * t1 * (0.5 + x1) + t2 * (0.5 + x2)) / 8;
  c->sk.b3 = t3 * (1 + x3 / 2) / 4;
  c->sk.b3p = t3 * (0.5 + x3) / 4;
  c->sk.b4 = d->W0 / 2;
  c->sk.b4p = d->W0 / 2;
  c->sk.alpha = d->alpha;
  c->sk.hb2m_n = d->hb2m_n;
  c->sk.hb2m_p = d->hb2m_p;
  c->sk.e2 = d->e2;
  c->last_sweeps = 0;
  c->fallbacks = 0;
  c->unconverged = 0;
  *out = c;
  return SKY_OK;
}

int sky_init_box(sky_ctx* c, const void* raw_n, const void* raw_p) {
  if (!c) return fail(SKY_ERR_INVALID, "null context");
  const void* raw[2] = {raw_n, raw_p};
  const int prec = c->d.precision == SKY_MIXED ? 1 : 0;
  if (!c->pc_ready) {   // learned preconditioner: initial network, Adam moments
    const Layout& L = c->lay;
    hipMemsetAsync(c->at(L.pc_M), 0, sizeof(float) * precond_nparams(), c->st);
    hipMemsetAsync(c->at(L.pc_V), 0, sizeof(float) * precond_nparams(), c->st);
    precond_init_params(c->at<float>(L.pc_P), 20161024u, c->st);
    precond_round(c->at<float>(L.pc_P), c->at<float>(L.pc_Pb), c->st);
    c->pc_ready = true;
  }
  c->prec = 0;   // the initial orthonormalisation runs in FP64 in both modes
  for (int q = 0; q < 2; ++q) {
    if (c->nq[q] == 0) continue;
    if (!raw[q]) return fail(SKY_ERR_INVALID, "null trial states");
    int rc = loewdin(c, q, raw[q], c->at(c->lay.psi[q]));
    if (rc) return rc;
    const size_t ne = size_t(c->nq[q]) * c->V;
    for (int t = 1; t < c->ntw; ++t)   // every twist starts from the same states
      hipMemcpyAsync(c->at(c->lay.psi[2 * t + q]), c->at(c->lay.psi[q]), ne * 16,
                     hipMemcpyDeviceToDevice, c->st);
    if (prec)
      for (int t = 0; t < c->ntw; ++t)
        convert_states(c->at(c->lay.psi[2 * t + q]), 0, c->at(c->lay.psi32[2 * t + q]), 1, ne,
                       c->st);
  }
  c->prec = prec;
  c->hpsi_lagged = false;
  fields(c);
  return hip_check(hipStreamSynchronize(c->st), "init");
}

int sky_apply_h(sky_ctx* c, int32_t q, const void* psi, void* hpsi, int32_t nstates,
                double* eps) {
  if (!c || q < 0 || q >= c->nset || !psi || !hpsi || nstates < 0)
    return fail(SKY_ERR_INVALID, "apply_h arguments");
  if (nstates > c->m_of(q)) return fail(SKY_ERR_INVALID, "apply_h: more states than the set holds");
  apply_h(c->n, c->prec, psi, hpsi, nstates, c->mfp(q), c->gset(q),
          eps ? c->at<double>(c->lay.tiles) : nullptr, eps, c->st, c->tune.lines);
  return hip_check(hipGetLastError(), "apply_h launch");
}

int sky_apply_h_noalloc(sky_ctx* c, int32_t q, const void* psi, void* hpsi, int32_t nstates,
                        double* eps) {
  if (!c || q < 0 || q >= c->nset || !psi || !hpsi || nstates < 0)
    return fail(SKY_ERR_INVALID, "apply_h_noalloc arguments");
  if (nstates > c->m_of(q))
    return fail(SKY_ERR_INVALID, "apply_h_noalloc: more states than the set holds");
  const size_t need = size_t(nstates) * size_t(grid_ntiles(c->n));
  if (need > noalloc_scratch_capacity())
    return fail(SKY_ERR_INVALID, "apply_h_noalloc: " + std::to_string(nstates) +
                                     " states need " + std::to_string(need) +
                                     " partial sums, more than the fixed scratch holds (" +
                                     std::to_string(noalloc_scratch_capacity()) + ")");
  double* part = nullptr;
  if (eps) {
    std::string err;
    if (noalloc_scratch(&part, &err)) return fail(SKY_ERR_HIP, err);
  }
  apply_h(c->n, c->prec, psi, hpsi, nstates, c->mfp(q), c->gset(q), part, eps, c->st,
          c->tune.lines);
  return hip_check(hipGetLastError(), "apply_h_noalloc launch");
}

int sky_damped_step(sky_ctx* c, int32_t q, const void* psi, const void* hpsi, const double* eps,
                    void* phi, int32_t nstates, double* r2) {
  if (!c || q < 0 || q >= c->nset || !psi || !hpsi || !eps || !phi || nstates < 0)
    return fail(SKY_ERR_INVALID, "damped_step arguments");
  if (nstates > c->m_of(q)) return fail(SKY_ERR_INVALID, "damped_step: more states than the set holds");
  double* r2o = r2 ? r2 : c->at<double>(c->lay.r2[q]);
  damped_step(c->n, c->prec, psi, hpsi, eps, phi, nstates, c->gset(q), c->d.damp_x0,
              c->d.damp_e0, c->hb2m(q), c->at<double>(c->lay.tiles), r2o, c->st, nullptr, nullptr,
              0, c->tune.damp_xy);
  return hip_check(hipGetLastError(), "damped_step launch");
}

int sky_orthonormalize(sky_ctx* c, int32_t q, const void* phi, const void* hphi, void* psi_out,
                       double* ritz) {
  if (!c || q < 0 || q >= c->nset || !phi || !psi_out)
    return fail(SKY_ERR_INVALID, "orthonormalize arguments");
  c->last_sweeps = 0;
  int rc = hphi ? rayleigh_ritz(c, q, phi, hphi, psi_out, ritz) : loewdin(c, q, phi, psi_out);
  if (rc) return rc;
  return hip_check(hipStreamSynchronize(c->st), "orthonormalize");
}

int sky_densities(sky_ctx* c) {
  if (!c) return fail(SKY_ERR_INVALID, "null context");
  fields(c);
  return hip_check(hipGetLastError(), "densities launch");
}

int sky_iterate(sky_ctx* c, int32_t max_iter, double tol, sky_report* rep) {
  if (!c || max_iter < 0) return fail(SKY_ERR_INVALID, "iterate arguments");
  hipStream_t st = c->st;
  std::vector<double> r2h;
  double de = 0.0;
  int it = 0, status = SKY_OK;
  c->fallbacks = 0;
  c->unconverged = 0;
  c->pc_iters = 0;
  const bool one_h = c->d.one_h != 0;
  for (; it < max_iter; ++it) {
    c->last_sweeps = 0;
    const bool learned = c->pc_on && c->pc_trained && c->pc_hold == 0;
    const bool lagged = one_h && c->hpsi_lagged;
    const int variant = (learned ? 1 : 0) | (lagged ? 2 : 0);
    for (int s = 0; s < c->nset; ++s) {
      if (c->m_of(s) == 0) continue;
      // step 2 and step 3a (graph segment A), steps 3b-3d on the host path,
      // step 3e (segment B)
      int rc = run_segment(c, c->graphs.a[s][variant], [&] { step_a(c, s, learned, lagged); });
      if (rc) return rc;
      rc = subspace_solve(c, s, c->at<double>(c->lay.ritz[s]));
      if (rc) return rc;
      rc = run_segment(c, c->graphs.b[s], [&] {
        if (one_h)
          subspace_combine(c, s, c->phi(s), c->psi(s), c->hphi(s), c->hpsi(s));
        else
          subspace_combine(c, s, c->phi(s), c->psi(s));
      });
      if (rc) return rc;
    }
    c->hpsi_lagged = one_h;
    // steps 4a, 4b, 5
    int rcf = run_segment(c, c->graphs.f, [&] { fields(c); });
    if (rcf) return rcf;
    // Delta-eps of the occupied states that entered this iteration (Eq. convergence)
    r2h.resize(size_t(c->nset) * std::max(c->nq[0], c->nq[1]));
    for (int s = 0; s < c->nset; ++s) {
      const int occ = c->nocc[s & 1];
      if (occ == 0) continue;
      int rc = hip_check(hipMemcpyAsync(r2h.data() + size_t(s) * std::max(c->nq[0], c->nq[1]),
                                        c->at(c->lay.r2[s]), sizeof(double) * occ,
                                        hipMemcpyDeviceToHost, st),
                         "r2 copy");
      if (rc) return rc;
    }
    int rcs = hip_check(hipStreamSynchronize(st), "iterate");
    if (rcs) return rcs;
    double sum = 0.0;
    for (int s = 0; s < c->nset; ++s)
      for (int a = 0; a < c->nocc[s & 1]; ++a)
        sum += r2h[size_t(s) * std::max(c->nq[0], c->nq[1]) + a];
    const int cnt = c->ntw * (c->nocc[0] + c->nocc[1]);
    t_flush(c);
    de = std::sqrt(sum / std::max(1, cnt));
    if (!std::isfinite(de)) return fail(SKY_ERR_NAN, "non-finite residual");
    // learned damping: back to the plain damping for PC_HOLD iterations when
    // the residual rose after a learned step
    if (c->pc_last && c->pc_rise >= 0.0 && c->de_prev >= 0.0 && de > (1.0 + c->pc_rise) * c->de_prev)
      c->pc_hold = PC_HOLD;
    else if (c->pc_hold > 0 && !learned) --c->pc_hold;
    c->pc_last = learned;
    c->pc_iters += learned ? 1 : 0;
    c->de_prev = de;
    // online training: fresh rows from both species (first twist), then a
    // few Adam steps
    if (c->pc_on && c->pc_every > 0 && ++c->pc_since >= c->pc_every) {
      c->pc_since = 0;
      for (int q = 0; q < 2; ++q) {
        if (c->nq[q] == 0) continue;
        int rc = pc_collect(c, q);
        if (rc) return rc;
      }
      pc_train(c, PC_RETRAIN_STEPS, c->pc_lr);
    }
    // precision ladder: finish in FP64 once the mixed form has done its part
    if (c->prec == 1 && c->d.ladder_tol > 0.0 && de <= c->d.ladder_tol) {
      for (int s = 0; s < c->nset; ++s)
        convert_states(c->at(c->lay.psi32[s]), 1, c->at(c->lay.psi[s]), 0,
                       size_t(c->m_of(s)) * c->V, st);
      c->prec = 0;
      c->hpsi_lagged = false;
      // launch shapes were tuned for the mixed kernels: the FP64 ones the
      // tuner found in its cache for this box, else the defaults, from here
      c->tune.lines = c->tune.lines64;
      c->tune.damp_xy = c->tune.damp64;
      c->tune.ovl[0] = c->tune.ovl64[0];
      c->tune.ovl[1] = c->tune.ovl64[1];
      fields(c);
      c->switched_at = c->iter_count + it + 1;
    }
    if (tol > 0.0 && de <= tol) { ++it; break; }
  }
  double e[8] = {0};
  int rc = hip_check(hipMemcpyAsync(e, c->at(c->lay.energy), sizeof(e), hipMemcpyDeviceToHost, st),
                     "energy copy");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(st), "iterate");
  if (rc) return rc;
  if (!std::isfinite(e[7])) return fail(SKY_ERR_NAN, "non-finite energy");
  if (tol > 0.0 && !(de <= tol)) status = SKY_NOT_CONVERGED;
  c->iter_count += it;
  if (rep) {
    rep->precision = c->prec ? SKY_MIXED : SKY_FP64;
    rep->iters = it;
    rep->residual = de;
    rep->energy = e[7];
    rep->energy_per_a = e[7] / double(std::max(1, c->nocc[0] + c->nocc[1]));
    rep->eig_iters = c->last_sweeps;
    rep->eig_fallbacks = c->fallbacks;
    rep->precond_iters = c->pc_iters;
    rep->eig_unconverged = c->unconverged;
  }
  return status;
}

int sky_get_view(sky_ctx* c, int32_t what, int32_t q, void** ptr, int64_t* count) {
  if (!c || !ptr || !count) return fail(SKY_ERR_INVALID, "get_view arguments");
  if (q < 0 || q >= c->nset) return fail(SKY_ERR_INVALID, "set index out of range");
  const int m = c->m_of(q);
  const int64_t st = int64_t(m) * c->V;
  switch (what) {
    case SKY_VIEW_PSI: *ptr = c->psi(q); *count = st; break;
    case SKY_VIEW_HPSI: *ptr = c->hpsi(q); *count = st; break;
    case SKY_VIEW_PHI: *ptr = c->phi(q); *count = st; break;
    case SKY_VIEW_HPHI: *ptr = c->hphi(q); *count = st; break;
    case SKY_VIEW_DENS: *ptr = c->at(c->lay.dens[q & 1]); *count = 11LL * c->n3; break;
    case SKY_VIEW_MEANFIELD: *ptr = c->at(c->lay.mf[q & 1]); *count = 5LL * c->n3; break;
    case SKY_VIEW_COULOMB: *ptr = c->at(c->lay.vc); *count = c->n3; break;
    case SKY_VIEW_ENERGY: *ptr = c->at(c->lay.energy); *count = 8; break;
    case SKY_VIEW_EPS: *ptr = c->at(c->lay.eps[q]); *count = m; break;
    case SKY_VIEW_RITZ: *ptr = c->at(c->lay.ritz[q]); *count = m; break;
    case SKY_VIEW_R2: *ptr = c->at(c->lay.r2[q]); *count = m; break;
    case SKY_VIEW_OVERLAP: *ptr = c->at(c->lay.matI); *count = int64_t(m) * m; break;
    case SKY_VIEW_HSUB: *ptr = c->at(c->lay.matH); *count = int64_t(m) * m; break;
    case SKY_VIEW_EVEC: *ptr = c->at(c->lay.matZ); *count = int64_t(m) * m; break;
    case SKY_VIEW_UMAT: *ptr = c->at(c->lay.matU); *count = int64_t(m) * m; break;
    case SKY_VIEW_PC_PARAMS: *ptr = c->at(c->lay.pc_P); *count = precond_nparams(); break;
    case SKY_VIEW_PC_GRAD: *ptr = c->at(c->lay.pc_G); *count = precond_nparams(); break;
    case SKY_VIEW_PC_SAMPLES: *ptr = c->at(c->lay.pc_S); *count = 6LL * PC_CAP; break;
    case SKY_VIEW_PC_GAINS: *ptr = c->at(c->lay.pc_gain); *count = int64_t(m) * PC_SHELLS; break;
    default: return fail(SKY_ERR_INVALID, "unknown view");
  }
  return SKY_OK;
}

int sky_set_states(sky_ctx* c, int32_t q, const void* psi, int32_t src_prec) {
  if (!c || q < 0 || q >= c->nset || !psi) return fail(SKY_ERR_INVALID, "set_states arguments");
  if (src_prec != SKY_FP64 && src_prec != SKY_MIXED)
    return fail(SKY_ERR_INVALID, "set_states: precision must be SKY_FP64 or SKY_MIXED");
  convert_states(psi, src_prec == SKY_MIXED ? 1 : 0, c->psi(q), c->prec, size_t(c->m_of(q)) * c->V,
                 c->st);
  c->hpsi_lagged = false;
  return hip_check(hipGetLastError(), "set_states");
}

int sky_get_states(sky_ctx* c, int32_t q, void* psi, int32_t dst_prec) {
  if (!c || q < 0 || q >= c->nset || !psi) return fail(SKY_ERR_INVALID, "get_states arguments");
  if (dst_prec != SKY_FP64 && dst_prec != SKY_MIXED)
    return fail(SKY_ERR_INVALID, "get_states: precision must be SKY_FP64 or SKY_MIXED");
  convert_states(c->psi(q), c->prec, psi, dst_prec == SKY_MIXED ? 1 : 0, size_t(c->m_of(q)) * c->V,
                 c->st);
  return hip_check(hipGetLastError(), "get_states");
}

int sky_get_iteration(sky_ctx* c, int64_t* iteration) {
  if (!c || !iteration) return fail(SKY_ERR_INVALID, "get_iteration arguments");
  *iteration = c->iter_count;
  return SKY_OK;
}

int sky_set_iteration(sky_ctx* c, int64_t iteration) {
  if (!c || iteration < 0) return fail(SKY_ERR_INVALID, "set_iteration arguments");
  c->iter_count = iteration;
  return SKY_OK;
}

int sky_set_timing(sky_ctx* c, int32_t enable) {
  if (!c) return fail(SKY_ERR_INVALID, "null context");
  int rc = hip_check(hipStreamSynchronize(c->st), "set_timing");
  if (rc) return rc;
  t_flush(c);
  c->timing = enable != 0;
  for (int p = 0; p < SKY_NPHASE; ++p)
    for (int q = 0; q < 2; ++q) { c->ms[p][q] = 0.0; c->cnt[p][q] = 0; }
  return SKY_OK;
}

int sky_get_timing(sky_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms) return fail(SKY_ERR_INVALID, "get_timing arguments");
  int rc = hip_check(hipStreamSynchronize(c->st), "get_timing");
  if (rc) return rc;
  t_flush(c);
  for (int p = 0; p < SKY_NPHASE; ++p)
    for (int q = 0; q < 2; ++q) {
      ms[2 * p + q] = c->ms[p][q];
      if (launches) launches[2 * p + q] = c->cnt[p][q];
    }
  return SKY_OK;
}

int sky_get_precision(sky_ctx* c, int32_t* precision) {
  if (!c || !precision) return fail(SKY_ERR_INVALID, "get_precision arguments");
  *precision = c->prec ? SKY_MIXED : SKY_FP64;
  return SKY_OK;
}

int sky_sync(sky_ctx* c) {
  if (!c) return fail(SKY_ERR_INVALID, "null context");
  return hip_check(hipStreamSynchronize(c->st), "sync");
}

const char* sky_last_error(void) { return g_err.c_str(); }

void sky_destroy(sky_ctx* c) {
  if (!c) return;
  hipStreamSynchronize(c->st);
  for (auto& m : c->marks) { hipEventDestroy(m.a); hipEventDestroy(m.b); }
  for (auto e : c->pool) hipEventDestroy(e);
  graphs_clear(c);
  delete c;
}

int sky_autotune(sky_ctx* c, const char* cache_path, sky_tuning* out) {
  if (!c) return fail(SKY_ERR_INVALID, "null context");
  hipStream_t st = c->st;
  int rc = hip_check(hipStreamSynchronize(st), "autotune");
  if (rc) return rc;
  auto kv = cache_read(cache_path);
  const char* pr = c->prec ? "mixed" : "fp64";
  const std::string klines = "h_lines/n" + std::to_string(c->n) + "/" + pr;
  const std::string kdamp = "damp_xy/n" + std::to_string(c->n) + "/" + pr;
  std::string kovl[2], ksq[2];
  for (int q = 0; q < 2; ++q) {
    kovl[q] = "overlap_split/m" + std::to_string(c->nq[q]) + "/k" + std::to_string(c->V) + "/" + pr;
    ksq[q] = "square_split/m" + std::to_string(c->nq[q]);
  }
  int timed = 0;
  if (c->prec) {   // FP64 shapes for a later ladder switch: cached entries only, not timed
    const std::string sn = "/n" + std::to_string(c->n) + "/fp64";
    int cand[4];
    const int nl = h_pass_lines(c->n, 0, cand);
    const int lv = cache_get(kv, "h_lines" + sn);
    c->tune.lines64 = 0;
    for (int i = 0; i < nl; ++i)
      if (cand[i] == lv) c->tune.lines64 = lv;
    const int dv = cache_has(kv, "damp_xy" + sn) ? cache_get(kv, "damp_xy" + sn) : -1;
    c->tune.damp64 = (dv == 0 || (dv == 1 && damp_slices_available(c->n, 0))) ? dv : -1;
    for (int q = 0; q < 2; ++q) {
      c->tune.ovl64[q] = 0;
      if (c->nq[q] == 0) continue;
      int oc[3];
      const int no = overlap_split_candidates(c->nq[q], c->V, oc);
      const int ov = cache_get(kv, "overlap_split/m" + std::to_string(c->nq[q]) + "/k" +
                                       std::to_string(c->V) + "/fp64");
      for (int i = 0; i < no; ++i)
        if (oc[i] == ov) c->tune.ovl64[q] = ov;
    }
  }
  // lines per workgroup of the h passes (species 0, or 1 if 0 is empty)
  {
    const int q = c->nq[0] > 0 ? 0 : 1;
    int v = cache_get(kv, klines);
    int cand[4];
    const int nl = h_pass_lines(c->n, c->prec, cand);
    bool ok = false;
    for (int i = 0; i < nl; ++i) ok = ok || cand[i] == v;
    if (!ok) {
      v = pick(st, cand, nl, [&](int lp) {
        apply_h(c->n, c->prec, c->psi(q), c->hpsi(q), c->nq[q], c->mfp(q), c->g, nullptr, nullptr,
                st, lp);
      });
      cache_put(kv, klines, v);
      ++timed;
    }
    c->tune.lines = v;
    // x and y transforms of the damped step on LDS slices (1) or by pencils (0)
    int dv = cache_has(kv, kdamp) ? cache_get(kv, kdamp) : -1;
    if (!damp_slices_available(c->n, c->prec)) dv = 0;   // pencils are the only variant
    if (dv != 0 && dv != 1) {
      const int dc[2] = {1, 0};
      const double hb = q ? c->d.hb2m_p : c->d.hb2m_n;
      double* eps = c->at<double>(c->lay.eps[q]);
      dv = pick(st, dc, 2, [&](int xy) {
        damped_step(c->n, c->prec, c->psi(q), c->hpsi(q), eps, c->phi(q), c->nq[q], c->g,
                    c->d.damp_x0, c->d.damp_e0, hb, c->at<double>(c->lay.tiles), nullptr, st,
                    nullptr, nullptr, 0, xy);
      });
      cache_put(kv, kdamp, dv);
      ++timed;
    }
    c->tune.damp_xy = dv;
  }
  for (int q = 0; q < 2; ++q) {
    const int m = c->nq[q];
    if (m == 0) continue;
    // overlap split-K
    int cand[3];
    const int nc = c->prec ? overlap_split_candidates_mixed(m, c->V, cand)
                           : overlap_split_candidates(m, c->V, cand);
    int v = cache_get(kv, kovl[q]);
    bool ok = false;
    for (int i = 0; i < nc; ++i) ok = ok || cand[i] == v;
    if (!ok) {
      void* I = c->at(c->lay.matI);
      void* H = c->at(c->lay.matH);
      if (c->prec) {
        unsigned int* mx = c->at<unsigned int>(c->lay.plS);
        plane_scale(c->psi(q), 0, size_t(m) * c->V, mx, st);
        split_planes_nt(c->psi(q), m, c->V, mx, c->at(c->lay.plA), st);
        v = pick(st, cand, nc, [&](int sp) {
          overlap_lower_planes(c->at(c->lay.plA), c->at(c->lay.plA), c->at(c->lay.plA), mx, mx, mx,
                               m, c->V, c->g.dV, I, H, c->at(c->lay.gemm_part), st, nullptr, sp);
        });
      } else {
        v = pick(st, cand, nc, [&](int sp) {
          overlap_lower(c->psi(q), c->psi(q), c->psi(q), m, c->V, c->g.dV, I, H,
                        c->at(c->lay.gemm_part), st, nullptr, sp);
        });
      }
      cache_put(kv, kovl[q], v);
      ++timed;
    }
    c->tune.ovl[q] = v;
    if (c->prec) {
      // waves per 128 x 128 tile of the overlap and recombination plane products
      const std::string kow = "plane_waves_overlap/m" + std::to_string(m) + "/k" + std::to_string(c->V);
      const std::string kcw = "plane_waves_combine/m" + std::to_string(m) + "/k" + std::to_string(c->V);
      const int wc[2] = {8, 4};
      unsigned int* mx = c->at<unsigned int>(c->lay.plS);
      int wv = cache_get(kv, kow);
      if (wv != 4 && wv != 8) {
        plane_scale(c->psi(q), 0, size_t(m) * c->V, mx, st);
        split_planes_nt(c->psi(q), m, c->V, mx, c->at(c->lay.plA), st);
        wv = pick(st, wc, 2, [&](int wz) {
          overlap_lower_planes(c->at(c->lay.plA), c->at(c->lay.plA), c->at(c->lay.plA), mx, mx, mx,
                               m, c->V, c->g.dV, c->at(c->lay.matI), c->at(c->lay.matH),
                               c->at(c->lay.gemm_part), st, nullptr, c->tune.ovl[q], wz);
        });
        cache_put(kv, kow, wv);
        ++timed;
      }
      c->tune.ovw[q] = wv;
      int cw = cache_get(kv, kcw);
      if (cw != 4 && cw != 8) {
        // any m x m transform times the states: the unit matrix's planes are
        // timed like any other
        identity(c->at(c->lay.matT), m, st);
        plane_scale(c->at(c->lay.matT), 1, size_t(m) * m, mx + 2, st);
        split_planes_t(c->at(c->lay.matT), 1, m, m, mx + 2, c->at(c->lay.plU), st);
        plane_scale(c->psi(q), 0, size_t(m) * c->V, mx, st);
        split_planes_t(c->psi(q), 0, m, c->V, mx, c->at(c->lay.plT), st);
        cw = pick(st, wc, 2, [&](int wz) {
          combine_planes(c->at(c->lay.plU), c->at(c->lay.plT), mx + 2, mx, c->phi(q), m, c->V, st,
                         wz);
        });
        cache_put(kv, kcw, cw);
        ++timed;
      }
      c->tune.cbw[q] = cw;
    }
    // square-product split-K
    int cs[4];
    const int ns = square_split_candidates(m, cs);
    v = cache_get(kv, ksq[q]);
    ok = false;
    for (int i = 0; i < ns; ++i) ok = ok || cs[i] == v;
    if (!ok) {
      v = pick(st, cs, ns, [&](int sp) {
        gemm_square(c->at(c->lay.matI), 1, c->at(c->lay.matH), 0, c->at(c->lay.matT), m, st,
                    c->at(c->lay.sq_part), 0, sp);
      });
      cache_put(kv, ksq[q], v);
      ++timed;
    }
    c->tune.sq[q] = v;
  }
  rc = hip_check(hipStreamSynchronize(st), "autotune runs");
  if (rc) return rc;
  c->tune.from_cache = timed == 0;
  if (timed && !cache_write(cache_path, kv)) return fail(SKY_ERR_INVALID, "cannot write the tuning cache");
  hipStreamSynchronize(c->st);
  graphs_clear(c);   // launch shapes may have changed
  return sky_get_tuning(c, out);
}

int sky_get_tuning(sky_ctx* c, sky_tuning* out) {
  if (!c) return fail(SKY_ERR_INVALID, "null context");
  if (!out) return SKY_OK;
  out->h_lines = c->tune.lines ? c->tune.lines : h_pass_default(c->n, c->prec);
  out->damp_xy = c->tune.damp_xy;
  for (int q = 0; q < 2; ++q) {
    out->overlap_split[q] = c->tune.ovl[q];
    out->square_split[q] = c->tune.sq[q];
    out->overlap_waves[q] = waves_of(c->tune.ovw[q]);
    out->combine_waves[q] = waves_of(c->tune.cbw[q]);
  }
  out->from_cache = c->tune.from_cache;
  return SKY_OK;
}

int sky_precond_collect(sky_ctx* c, int32_t q, int32_t* total) {
  if (!c || q < 0 || q >= c->nset) return fail(SKY_ERR_INVALID, "precond_collect arguments");
  int rc = pc_collect(c, q);
  if (rc) return rc;
  if (total) *total = c->pc_count;
  return SKY_OK;
}

int sky_precond_loss_grad(sky_ctx* c, int32_t nsamples, double* loss) {
  if (!c || nsamples < 1 || nsamples > PC_CAP) return fail(SKY_ERR_INVALID, "precond_loss_grad arguments");
  const int keep = c->pc_count;
  c->pc_count = nsamples;
  const double w = precond_wsum(c);
  precond_round(c->at<float>(c->lay.pc_P), c->at<float>(c->lay.pc_Pb), c->st);
  const double l = precond_pass(c, w, 1);
  c->pc_count = keep;
  if (loss) *loss = l;
  return hip_check(hipStreamSynchronize(c->st), "precond_loss_grad");
}

int sky_precond_train(sky_ctx* c, int32_t steps, double lr, double* loss) {
  if (!c || steps < 1 || !(lr > 0.0)) return fail(SKY_ERR_INVALID, "precond_train arguments");
  if (c->pc_count < 1) return fail(SKY_ERR_INVALID, "precond_train: no samples collected");
  const double l = pc_train(c, steps, lr);
  if (loss) *loss = l;
  return hip_check(hipStreamSynchronize(c->st), "precond_train");
}

int sky_precond_set_rows(sky_ctx* c, int32_t nrows) {
  if (!c || nrows < 0 || nrows > PC_CAP) return fail(SKY_ERR_INVALID, "precond_set_rows arguments");
  c->pc_count = nrows;
  c->pc_wr = nrows;
  return SKY_OK;
}

int sky_precond_use(sky_ctx* c, int32_t enable, double rise_tol, int32_t retrain_every) {
  if (!c || !std::isfinite(rise_tol) || retrain_every < 0)
    return fail(SKY_ERR_INVALID, "precond_use arguments");
  if (enable && !c->pc_trained) return fail(SKY_ERR_INVALID, "precond_use: the network is not trained");
  c->pc_on = enable != 0;
  c->pc_rise = rise_tol;
  c->pc_every = retrain_every;
  c->pc_since = 0;
  c->pc_hold = 0;
  c->pc_last = false;
  c->de_prev = -1.0;
  return SKY_OK;
}

int sky_set_preconditioner(sky_ctx* c, const float* params, int32_t nparams) {
  if (!c || !params) return fail(SKY_ERR_INVALID, "set_preconditioner arguments");
  if (nparams != precond_nparams())
    return fail(SKY_ERR_INVALID, "set_preconditioner: parameter count differs from the network's");
  const Layout& L = c->lay;
  const size_t bytes = sizeof(float) * size_t(nparams);
  hipMemcpyAsync(c->at(L.pc_P), params, bytes, hipMemcpyDeviceToDevice, c->st);
  zero_f32(c->at<float>(L.pc_M), size_t(nparams), c->st);
  zero_f32(c->at<float>(L.pc_V), size_t(nparams), c->st);
  precond_round(c->at<float>(L.pc_P), c->at<float>(L.pc_Pb), c->st);
  c->pc_step = 0;
  c->pc_ready = true;
  c->pc_trained = true;
  return hip_check(hipStreamSynchronize(c->st), "set_preconditioner");
}

int sky_set_graphs(sky_ctx* c, int32_t enable) {
  if (!c) return fail(SKY_ERR_INVALID, "null context");
  if (enable && !c->st) return fail(SKY_ERR_INVALID, "graph capture needs a stream other than the null stream");
  int rc = hip_check(hipStreamSynchronize(c->st), "set_graphs");
  if (rc) return rc;
  graphs_clear(c);
  c->graphs.on = enable != 0;
  return SKY_OK;
}

int sky_iterate_graph(sky_ctx* c, int32_t max_iter, double tol, int32_t chunk, sky_report* rep) {
  if (!c || max_iter < 0 || chunk < 1) return fail(SKY_ERR_INVALID, "iterate_graph arguments");
  if (!dev_iteration_ok(c)) return sky_iterate(c, max_iter, tol, rep);
  DevRun r;
  r.c = c;
  r.max_iter = max_iter;
  r.chunk = chunk;
  r.tol = tol;
  int rc = dev_start(r);
  if (rc) return rc;
  while (!r.finished) {
    rc = dev_launch(r);
    if (rc) return rc;
    rc = dev_collect(r);
    if (rc) return rc;
  }
  return dev_finish(r, rep);
}

int sky_batch_iterate_graph(sky_ctx* const* ctxs, int32_t nbox, int32_t nthreads,
                            int32_t max_iter, double tol, int32_t chunk, sky_report* reps,
                            int32_t* status) {
  if (!ctxs || nbox < 1 || nthreads < 1 || max_iter < 0 || chunk < 1 || !reps || !status)
    return fail(SKY_ERR_INVALID, "batch_iterate_graph arguments");
  for (int i = 0; i < nbox; ++i) {
    if (!ctxs[i]) return fail(SKY_ERR_INVALID, "batch_iterate_graph: null context");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(SKY_ERR_INVALID, "batch_iterate_graph: a context appears twice");
  }
  int dev = 0;
  int rc = hip_check(hipGetDevice(&dev), "batch_iterate_graph");
  if (rc) return rc;
  rc = hip_check(hipDeviceSynchronize(), "batch_iterate_graph");
  if (rc) return rc;
  // the same longest-processing-time assignment as sky_batch_iterate
  const int nw = std::min(nthreads, nbox);
  std::vector<std::pair<double, int>> cost(nbox);
  for (int i = 0; i < nbox; ++i) {
    const sky_ctx* c = ctxs[i];
    double w = 0.0;
    for (int q = 0; q < 2; ++q)
      w += double(c->ntw) * double(c->nq[q]) * double(c->V) *
           (double(c->nq[q]) + 40.0 * std::log2(double(c->V)));
    cost[i] = {w, i};
  }
  std::sort(cost.begin(), cost.end(), [](auto& x, auto& y) { return x.first > y.first; });
  std::vector<std::vector<int>> mine(nw);
  std::vector<double> load(nw, 0.0);
  for (auto& [w, i] : cost) {
    const int k = int(std::min_element(load.begin(), load.end()) - load.begin());
    mine[k].push_back(i);
    load[k] += w;
  }
  std::vector<std::string> errs(nw);
  // each worker drives its boxes round by round: every unfinished box gets a
  // chunk of captured iterations queued on the worker's stream, then one
  // drain of the stream and one read of every box's flags
  auto worker = [&](int k) {
    hipSetDevice(dev);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (int i : mine[k]) status[i] = SKY_ERR_HIP;
      errs[k] = "batch_iterate_graph: stream creation failed";
      return;
    }
    std::vector<DevRun> runs(mine[k].size());
    std::vector<hipStream_t> keep(mine[k].size());
    std::vector<bool> keep_graphs(mine[k].size());
    std::vector<bool> dev_ok(mine[k].size());
    for (size_t b = 0; b < mine[k].size(); ++b) {
      const int i = mine[k][b];
      sky_ctx* c = ctxs[i];
      keep[b] = c->st;
      keep_graphs[b] = c->graphs.on;
      c->st = s;
      c->graphs.on = true;
      std::memset(&reps[i], 0, sizeof(sky_report));
      dev_ok[b] = dev_iteration_ok(c);
      if (!dev_ok[b]) {   // host-decided options: the host path, box by box
        status[i] = sky_iterate(c, max_iter, tol, &reps[i]);
        runs[b].finished = true;
        continue;
      }
      runs[b].c = c;
      runs[b].max_iter = max_iter;
      runs[b].chunk = chunk;
      runs[b].tol = tol;
      status[i] = dev_start(runs[b]);
      if (status[i]) runs[b].finished = true;
    }
    for (;;) {
      bool any = false;
      for (size_t b = 0; b < runs.size(); ++b) {
        if (runs[b].finished || !dev_ok[b]) continue;
        any = true;
        const int rc = dev_launch(runs[b]);
        if (rc) { status[mine[k][b]] = rc; runs[b].finished = true; }
      }
      if (!any) break;
      for (size_t b = 0; b < runs.size(); ++b) {
        if (runs[b].finished || !dev_ok[b]) continue;
        const int rc = dev_collect(runs[b]);
        if (rc) { status[mine[k][b]] = rc; runs[b].finished = true; runs[b].status = rc; }
      }
    }
    for (size_t b = 0; b < runs.size(); ++b) {
      const int i = mine[k][b];
      sky_ctx* c = ctxs[i];
      if (dev_ok[b] && status[i] == SKY_OK) status[i] = dev_finish(runs[b], &reps[i]);
      if (status[i] != SKY_OK && status[i] != SKY_NOT_CONVERGED && errs[k].empty()) errs[k] = g_err;
      hipStreamSynchronize(s);
      c->graphs.on = keep_graphs[b];
      c->st = keep[b];
    }
    hipStreamDestroy(s);
  };
  std::vector<std::thread> pool;
  for (int k = 1; k < nw; ++k) pool.emplace_back(worker, k);
  worker(0);
  for (auto& t : pool) t.join();
  for (int i = 0; i < nbox; ++i)
    if (status[i] != SKY_OK && status[i] != SKY_NOT_CONVERGED) {
      std::string msg;
      for (auto& e : errs) if (!e.empty()) { msg = e; break; }
      return fail(status[i], "batch_iterate_graph: box " + std::to_string(i) + ": " + msg);
    }
  return SKY_OK;
}

int sky_batch_iterate(sky_ctx* const* ctxs, int32_t nbox, int32_t nthreads, int32_t max_iter,
                      double tol, sky_report* reps, int32_t* status) {
  if (!ctxs || nbox < 1 || nthreads < 1 || max_iter < 0 || !reps || !status)
    return fail(SKY_ERR_INVALID, "batch_iterate arguments");
  for (int i = 0; i < nbox; ++i) {
    if (!ctxs[i]) return fail(SKY_ERR_INVALID, "batch_iterate: null context");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(SKY_ERR_INVALID, "batch_iterate: a context appears twice");
  }
  int dev = 0;
  int rc = hip_check(hipGetDevice(&dev), "batch_iterate");
  if (rc) return rc;
  // work issued earlier on the contexts' own streams completes first
  rc = hip_check(hipDeviceSynchronize(), "batch_iterate");
  if (rc) return rc;
  // longest-processing-time assignment of boxes to workers by the cost of an
  // iteration: the subspace products (m^2 V) and the FFT passes (m V log V)
  const int nw = std::min(nthreads, nbox);
  std::vector<std::pair<double, int>> cost(nbox);
  for (int i = 0; i < nbox; ++i) {
    const sky_ctx* c = ctxs[i];
    double w = 0.0;
    for (int q = 0; q < 2; ++q)
      w += double(c->ntw) * double(c->nq[q]) * double(c->V) *
           (double(c->nq[q]) + 40.0 * std::log2(double(c->V)));
    cost[i] = {w, i};
  }
  std::sort(cost.begin(), cost.end(), [](auto& x, auto& y) { return x.first > y.first; });
  std::vector<std::vector<int>> mine(nw);
  std::vector<double> load(nw, 0.0);
  for (auto& [w, i] : cost) {
    const int k = int(std::min_element(load.begin(), load.end()) - load.begin());
    mine[k].push_back(i);
    load[k] += w;
  }
  std::vector<std::string> errs(nw);
  auto worker = [&](int k) {
    hipSetDevice(dev);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (int i : mine[k]) status[i] = SKY_ERR_HIP;
      errs[k] = "batch_iterate: stream creation failed";
      return;
    }
    for (int i : mine[k]) {
      sky_ctx* c = ctxs[i];
      hipStream_t keep = c->st;
      const bool keep_graphs = c->graphs.on;
      c->st = s;
      c->graphs.on = true;
      std::memset(&reps[i], 0, sizeof(sky_report));
      status[i] = sky_iterate(c, max_iter, tol, &reps[i]);
      if (status[i] != SKY_OK && status[i] != SKY_NOT_CONVERGED && errs[k].empty()) errs[k] = g_err;
      hipStreamSynchronize(s);
      c->graphs.on = keep_graphs;
      c->st = keep;
    }
    hipStreamDestroy(s);
  };
  std::vector<std::thread> pool;
  for (int k = 1; k < nw; ++k) pool.emplace_back(worker, k);
  worker(0);
  for (auto& t : pool) t.join();
  for (int i = 0; i < nbox; ++i)
    if (status[i] != SKY_OK && status[i] != SKY_NOT_CONVERGED) {
      std::string msg;
      for (auto& e : errs) if (!e.empty()) { msg = e; break; }
      return fail(status[i], "batch_iterate: box " + std::to_string(i) + ": " + msg);
    }
  return SKY_OK;
}

}  // extern "C"
