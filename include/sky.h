/*
 * sky.h - C ABI of the MI355X (gfx950) damped-gradient Skyrme solver.
 *
 * One static iteration of nuclear DFT on an equidistant periodic grid, as in
 * Afibuzzaman, Schuetrumpf & Aktulga, "Scalable Nuclear Density Functional
 * Theory with Sky3D" (Sec. 2, Fig. 1): h*psi with FFT derivatives, the
 * damped gradient step (Eq. dampstep), overlap and subspace-Hamiltonian
 * matrices (Eqs. normmatrix, hammatrix), orthonormalisation plus
 * diagonalisation (Sec. 3.3.2-3.3.3), densities (Eqs. rho, curr, tau) and
 * the Skyrme + Coulomb mean field (Eq. Skyrme, Sec. 2.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Precision (sky_box_desc.precision): SKY_FP64 keeps every state in
 *   complex128 and every operation in binary64.  SKY_MIXED keeps the states
 *   in complex64, runs FFTs and h*psi in binary32, forms the overlap,
 *   subspace-Hamiltonian and recombination products from a two-term FP16
 *   split (one power-of-two scale per operand matrix) on the matrix cores
 *   with FP32 accumulation folded into FP64, and
 *   keeps the Cholesky, eigensolver, densities, mean field and energy sums
 *   in binary64.  Reductions (<h>, residuals, densities) are binary64 in both
 *   modes.  State pointers passed to the per-step calls must have the
 *   context's current precision (sky_get_precision): complex128 or complex64.
 *   Fields and subspace matrices are always binary64 / complex128.
 * - State layout: [state][spin][z][y][x], x fastest, spin 0 = up.  One state
 *   of species q holds V = 2*n^3 complex values.  Field layout: [z][y][x].
 * - Grid: cubic, n points per axis, n in {8, 16, 24, 32, 48, 64}, spacing dx
 *   (fm), periodic; point i sits at i*dx.
 * - Pointers named *_dev are device pointers on the device that is current
 *   when sky_create is called; host pointers are named otherwise.  The caller
 *   owns every buffer it passes in.  All bulk device memory of a context lives
 *   in the caller's workspace (sky_workspace_size / sky_create); the library
 *   allocates no device memory of its own and never frees caller memory.
 * - Streams: every call enqueues its work on the stream given to sky_create
 *   and returns without waiting, except sky_init_box, sky_orthonormalize and
 *   sky_iterate, which wait for the stream (they read small results on the
 *   host: convergence norms, particle number, residuals).
 * - Errors: functions return SKY_OK (0) or a positive status on success and
 *   a negative SKY_ERR_* code on failure; sky_last_error() then describes the
 *   failure (per host thread).  No C++ exception crosses this interface.
 * - Thread safety: one context per host thread; concurrent calls on one
 *   context are not allowed.
 */
#ifndef SKY_H
#define SKY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SKY_OK = 0,
  SKY_NOT_CONVERGED = 1,            /* sky_iterate: max_iter reached above tol  */
  SKY_ERR_INVALID = -1,             /* bad argument                             */
  SKY_ERR_UNSUPPORTED_GRID = -2,    /* n not in {8,16,24,32,48,64}              */
  SKY_ERR_WORKSPACE = -3,           /* workspace too small or misaligned        */
  SKY_ERR_HIP = -4,                 /* a HIP runtime call failed                */
  SKY_ERR_NOT_POSITIVE_DEFINITE = -5, /* overlap matrix not positive definite   */
  SKY_ERR_NAN = -6                  /* non-finite residual or energy            */
};

enum { SKY_NEUTRON = 0, SKY_PROTON = 1 };
enum { SKY_FP64 = 0, SKY_MIXED = 1 };
/* Subspace update of Fig. 1 steps 3b-3e (sky_box_desc.update). */
enum {
  SKY_UPDATE_EXACT = 0,   /* generalised Rayleigh-Ritz: psi = phi C Z with C^H I C = 1 */
                          /* and Z the eigenvectors of H' = C^H H C                */
  SKY_UPDATE_PAPER = 1    /* Sec. 3.3.3 as printed: Z from H alone (3b), C = I^-1/2  */
                          /* from I alone (3c), psi = phi Z C (3d-3e)                */
};
#define SKY_MAX_TWIST 32

/* Box, force and damping of one solve.  Skyrme parameters in the usual
 * units: t0 MeV fm^3, t1 t2 MeV fm^5, t3 MeV fm^(3+3 alpha), W0 MeV fm^5,
 * hb2m_* = hbar^2/2m in MeV fm^2, e2 = e^2 in MeV fm (0 switches Coulomb
 * off).  damp_x0 is the step delta and damp_e0 the energy E0 (MeV) of the
 * damping operator delta / (T + E0) of Eq. dampstep. */
typedef struct {
  int32_t n;                        /* grid points per axis                     */
  double dx;                        /* grid spacing, fm                         */
  int32_t n_neutrons, n_protons;    /* occupied states per species (v^2 = 1)    */
  double t0, t1, t2, t3, x0, x1, x2, x3, alpha, W0;
  double hb2m_n, hb2m_p, e2;
  double damp_x0, damp_e0;
  int32_t precision;                /* SKY_FP64 or SKY_MIXED                    */
  double ladder_tol;                /* SKY_MIXED: switch to FP64 once Delta-eps */
                                    /* <= ladder_tol (MeV); <= 0 never          */
  /* Sec. 2.1: occupations v^2 in {0, 1}, more wave functions than particles
   * allowed.  Each species carries extra_q states beyond its n_q particles;
   * after every subspace update the states are in ascending order of their
   * subspace eigenvalues and the first n_q are occupied (aufbau).  Only the
   * occupied states enter the densities and Delta-eps. */
  int32_t extra_n, extra_p;
  /* Sec. 1, twist-averaged boundary conditions: ntwist (<= 1: one twist)
   * Bloch phases theta (radians per axis x, y, z; all 0 = periodic).  Every
   * twist carries its own n_q + extra_q states of each species; the
   * derivatives of a state of twist t are d_m + i theta_m / L; one mean field,
   * built from the densities averaged over the twists, serves all of them.
   * The energy is the functional of the averaged densities. */
  int32_t ntwist;
  double twist[SKY_MAX_TWIST][3];
  int32_t update;                   /* SKY_UPDATE_EXACT or SKY_UPDATE_PAPER     */
  /* one_h != 0: one h application per iteration.  Sec. 3.4 keeps h psi
   * (hampsi) for step 3a; here the h phi of step 3a is carried through the
   * subspace update, h psi_new = (h phi) U, and the next gradient step uses
   * it, i.e. the Hamiltonian of the previous mean field, with
   * <psi|h psi> = the subspace eigenvalues.  Same fixed point, one FFT
   * application fewer, one combination product more.  Needs
   * SKY_UPDATE_EXACT. */
  int32_t one_h;
  /* Refinement steps of the device-decided iteration (sky_iterate_graph)
   * before it hands the set to the host path: 0 = the default (4), else
   * 1..39. */
  int32_t dev_refine_steps;
} sky_box_desc;

typedef struct {
  int32_t iters;          /* iterations performed by this call                 */
  double residual;        /* Delta-eps (MeV, Eq. convergence) of the states     */
                          /* entering the last iteration                        */
  double energy;          /* total energy after the last iteration, MeV         */
  double energy_per_a;    /* energy / (N + Z)                                   */
  int32_t eig_iters;      /* subspace eigensolver iterations of the last        */
                          /* iteration (n + p): refinement steps, or Jacobi     */
                          /* sweeps where the refinement fell back              */
  int32_t precision;      /* precision of the states after the call             */
  int32_t eig_fallbacks;  /* subspace eigensolves of this call that fell back   */
                          /* from the refinement to the Jacobi solver           */
  int32_t precond_iters;  /* iterations of this call whose damped step used     */
                          /* the learned gains (sky_precond_use)                */
  int32_t eig_unconverged;  /* subspace eigensolves of this call that stopped    */
                            /* at the Jacobi solver's sweep limit above its      */
                            /* tolerance (the result is then not exact Ritz     */
                            /* vectors)                                          */
} sky_report;

/* Views into the context's device buffers (sky_get_view).  State sets: the
 * argument q of the per-species calls and views is a set index, set
 * q = 2 t + s holding species s (0 = n, 1 = p) of twist t; without twists
 * it is the species.  A set holds n_s + extra_s states.  Field views
 * (DENS, MEANFIELD) take the species q & 1; PHI, HPHI and the subspace
 * matrices are shared by the sets of a species (or of both) and hold the
 * set last processed. */
enum {
  SKY_VIEW_PSI = 0,       /* orthonormal states of species q, [n_q][2][n^3]      */
                          /* (complex128, or complex64 in mixed precision)      */
  SKY_VIEW_HPSI = 1,      /* h psi of the last iteration                         */
  SKY_VIEW_PHI = 2,       /* damped (non-orthonormal) states                     */
  SKY_VIEW_HPHI = 3,      /* h phi                                              */
  SKY_VIEW_DENS = 4,      /* 11 fields rho,tau,Jx,Jy,Jz,sx,sy,sz,jx,jy,jz [n^3]  */
  SKY_VIEW_MEANFIELD = 5, /* 5 fields U,B,Wx,Wy,Wz of species q [n^3] f64        */
  SKY_VIEW_COULOMB = 6,   /* Coulomb potential [n^3] f64 (q ignored)             */
  SKY_VIEW_ENERGY = 7,    /* 8 f64: kin, rho, rho^(2+a), rho*tau, rho*lap rho,   */
                          /* spin-orbit, Coulomb, total (MeV) (q ignored)        */
  SKY_VIEW_EPS = 8,       /* Rayleigh quotients <psi|h|psi> of species q [n_q]   */
  SKY_VIEW_RITZ = 9,      /* ascending subspace eigenvalues of species q [n_q]   */
  SKY_VIEW_R2 = 10,       /* ||h psi - eps psi||^2 of species q [n_q]            */
  /* Subspace matrices of the last sky_orthonormalize / iteration, complex128
   * [n_q][n_q] row-major, valid for the species q of that call:          */
  SKY_VIEW_OVERLAP = 11,  /* I = <phi|phi> (Eq. normmatrix)                      */
  SKY_VIEW_HSUB = 12,     /* H = <phi|h phi> (Eq. hammatrix); unset by Loewdin   */
  SKY_VIEW_EVEC = 13,     /* eigenvectors (columns) of H' (or of I for Loewdin)  */
  SKY_VIEW_UMAT = 14,     /* combined transform U, psi = phi U                   */
  SKY_VIEW_PC_PARAMS = 15,  /* learned damping: FP32 master parameters [P] (f32)   */
  SKY_VIEW_PC_GRAD = 16,    /* gradient of the last loss evaluation [P] (f32)      */
  SKY_VIEW_PC_SAMPLES = 17, /* sample rows [16384][6] f32: 4 features, target     */
                            /* gain, weight (sky_precond_collect fills them)       */
  SKY_VIEW_PC_GAINS = 18    /* gains [n_q][8] of the last learned step (f32)       */
};

/* Timed phases of one iteration (sky_set_timing / sky_get_timing). */
enum {
  SKY_PHASE_APPLY_H = 0,       /* h psi and h phi (Fig. 1 step 2)                 */
  SKY_PHASE_DAMP = 1,          /* damped gradient step (Eq. dampstep)             */
  SKY_PHASE_OVERLAP_GEMM = 2,  /* the I/H GEMM kernel alone (step 3a)             */
  SKY_PHASE_SUBSPACE = 3,      /* I/H reduction, Cholesky, H', eigensolver, U     */
  SKY_PHASE_COMBINE_GEMM = 4,  /* psi = phi U GEMM kernel (step 3e)               */
  SKY_PHASE_DENSITIES = 5,     /* rho, tau, J (step 4a)                           */
  SKY_PHASE_MEANFIELD = 6,     /* mean field, Coulomb, energy (steps 4b, 5)       */
  SKY_PHASE_SPLIT = 7,         /* FP16 split planes of phi, h phi (mixed only)    */
  SKY_NPHASE = 8
};

typedef struct sky_ctx sky_ctx;

/* Bytes of device workspace a context for `d` needs (256-byte aligned). */
int sky_workspace_size(const sky_box_desc* d, size_t* bytes);

/* Create a context.  workspace_dev: caller-owned device buffer of at least
 * sky_workspace_size bytes, 256-byte aligned, alive until sky_destroy.
 * stream: hipStream_t (NULL = the default stream).  Errors: INVALID,
 * UNSUPPORTED_GRID, WORKSPACE. */
int sky_create(const sky_box_desc* d, void* workspace_dev, size_t bytes, void* stream,
               sky_ctx** out);

/* Fig. 1 step 1 (Sec. 2.2: trial plane waves for periodic systems): take
 * caller trial states raw_n_dev [n_neutrons + extra_n][2][n^3] and raw_p_dev
 * [n_protons + extra_p][2][n^3] (complex128 in both precisions, need not be
 * orthonormal; read only), orthonormalise them in binary64 by Loewdin's
 * C = I^(-1/2) (Eqs. Loewedin, orthmatvec), give every twist the same
 * states, round them to complex64 under SKY_MIXED, then build densities
 * (the first n_q states of each species occupied), mean field and energy.
 * Waits for the stream.
 * Errors: INVALID, NOT_POSITIVE_DEFINITE (linearly dependent states: an
 * overlap eigenvalue at or below 1e-10), NAN, HIP. */
int sky_init_box(sky_ctx* c, const void* raw_n_dev, const void* raw_p_dev);

/* h psi for `nstates` states of set q (species q & 1, twist q >> 1: its
 * derivatives carry that twist's Bloch shift) with the context's current mean
 * field (Sec. 2.2: kinetic + Skyrme + Coulomb, FFT derivatives):
 *   h psi = U psi - sum_m d_m(B d_m psi) + (i/2) sum_m [A_m d_m psi + d_m(A_m psi)],
 *   A_m = (W x sigma)_m.
 * psi_dev, hpsi_dev: [nstates][2][n^3] c128, must not overlap.  eps_dev (may
 * be NULL): receives Re <psi|h psi> per state (f64, nstates).  Asynchronous. */
int sky_apply_h(sky_ctx* c, int32_t q, const void* psi_dev, void* hpsi_dev, int32_t nstates,
                double* eps_dev);

/* sky_apply_h for callers that cannot allocate device memory or take it
 * from a workspace per call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same kernels and results
 * (bit for bit), with the per-workgroup partial sums of <psi|h psi> held in
 * a fixed device array of the library (8 MiB, one per device, kept until the
 * process ends; its address is looked up once per device, on the first call
 * there) instead of the context's workspace.  It calls no allocating
 * routine.  Every call on one device shares that array and the partials are
 * overwritten in full by each call (nothing needs clearing), so calls that
 * overlap in time on one device race: issue them on one stream, or order
 * them.  Limit: nstates x (grid tiles of one pass; 144 at n = 48, 256 at
 * n = 64) partial sums must fit the array's 2^20 doubles, else
 * SKY_ERR_INVALID with the sizes in the message.  Errors: INVALID, HIP. */
int sky_apply_h_noalloc(sky_ctx* c, int32_t q, const void* psi_dev, void* hpsi_dev,
                        int32_t nstates, double* eps_dev);

/* Damped gradient step, Eq. dampstep:
 *   phi = psi - x0 F^-1[ F(h psi - eps psi) / (E0 + hb2m_q |k|^2) ],
 * eps_dev: <psi|h psi> per state (from sky_apply_h).  r2_dev (f64, nstates)
 * receives ||h psi - eps psi||^2, the per-state term of Eq. convergence.
 * phi_dev must not overlap psi_dev or hpsi_dev.  Asynchronous. */
int sky_damped_step(sky_ctx* c, int32_t q, const void* psi_dev, const void* hpsi_dev,
                    const double* eps_dev, void* phi_dev, int32_t nstates, double* r2_dev);

/* Orthonormalise (and diagonalise) the n_q states phi_dev of species q into
 * psi_out_dev (must not overlap phi_dev).
 * hphi_dev != NULL: Sec. 3.3.2-3.3.3 as a generalised Rayleigh-Ritz step:
 *   I = <phi|phi>, H = <phi|h phi> (lower triangles, Fig. 3), I = L L^H,
 *   H' = L^-1 H L^-H = Z diag(lam) Z^H (ascending), psi = phi (L^-H Z);
 *   ritz_dev (may be NULL) receives lam (f64, n_q).
 * hphi_dev == NULL: Loewdin, psi = phi I^(-1/2).
 * Waits for the stream.  Errors: NOT_POSITIVE_DEFINITE (a Cholesky pivot at
 * or below 1e-10), NAN (a non-finite overlap), HIP. */
int sky_orthonormalize(sky_ctx* c, int32_t q, const void* phi_dev, const void* hphi_dev,
                       void* psi_out_dev, double* ritz_dev);

/* Fig. 1 steps 4a-4b and the energy: densities rho, tau, J (+ spin and
 * current diagnostics) of the context's current states of both species
 * (Eqs. rho, curr, tau with v^2 = 1), mean fields U, B, W, the Coulomb
 * potential and the total energy.  Asynchronous. */
int sky_densities(sky_ctx* c);

/* Run up to max_iter damped-gradient iterations (Fig. 1 steps 2-5) on the
 * context's states.  Under SKY_MIXED with ladder_tol > 0 the context switches
 * itself to binary64 states after the first iteration whose Delta-eps is
 * <= ladder_tol and continues in FP64 (the precision ladder).  tol_mev > 0: stop once Delta-eps <= tol_mev (returns
 * SKY_OK), else SKY_NOT_CONVERGED after max_iter; tol_mev <= 0: run exactly
 * max_iter iterations.  Delta-eps runs over the occupied states of every
 * set.  report (host, may be NULL) is filled.  Waits for the stream.
 * Errors: NAN (a non-finite overlap, subspace matrix, residual or energy),
 * NOT_POSITIVE_DEFINITE (linearly dependent damped states), HIP. */
int sky_iterate(sky_ctx* c, int32_t max_iter, double tol_mev, sky_report* report);

/* Device pointer and element count (complex or f64 elements, see SKY_VIEW_*)
 * of one of the context's buffers.  The memory stays owned by the caller's
 * workspace. */
int sky_get_view(sky_ctx* c, int32_t what, int32_t q, void** ptr_dev, int64_t* count);

/* Fig. 1 step 6 and its inverse: state I/O for checkpoint and resume.
 * sky_set_states copies the n_q + extra_q states of set q from psi_dev
 * ([states][2][n^3], complex128 when src_precision is SKY_FP64, complex64
 * when SKY_MIXED; read only) into the context, rounding or widening to the
 * context's current precision.  The states are taken as they are (they are
 * expected orthonormal and, with extra states, in ascending order of their
 * eigenvalues); call sky_densities afterwards to rebuild the mean field
 * from them.  Asynchronous.  With the same states, iteration counter and
 * settings, sky_iterate then continues the FP64 trajectory bit for bit.
 * sky_get_states copies them out the same way (dst_precision).
 * Errors: INVALID (set index, null pointer, precision). */
int sky_set_states(sky_ctx* c, int32_t q, const void* psi_dev, int32_t src_precision);
int sky_get_states(sky_ctx* c, int32_t q, void* psi_dev, int32_t dst_precision);

/* Iterations run on this context (sky_iterate adds to it; the online
 * retraining cadence of the learned damping and the precision-ladder record
 * count from it).  A resumed run sets the counter of its checkpoint. */
int sky_get_iteration(sky_ctx* c, int64_t* iteration);
int sky_set_iteration(sky_ctx* c, int64_t iteration);

/* Phase timing of sky_iterate: enable != 0 starts recording HIP event pairs
 * on the context stream around every phase (and resets the accumulators);
 * enable == 0 stops.  Waits for the stream. */
int sky_set_timing(sky_ctx* c, int32_t enable);

/* Accumulated device time (ms) and number of timed launches per phase and
 * species since sky_set_timing: ms[2*phase + q], launches[2*phase + q]
 * (host arrays of 2*SKY_NPHASE; launches may be NULL; phases that are not
 * per species use q = 0).  Waits for the stream. */
int sky_get_timing(sky_ctx* c, double* ms, int64_t* launches);

/* Current precision of the context's states (SKY_FP64 or SKY_MIXED). */
int sky_get_precision(sky_ctx* c, int32_t* precision);

/* Launch shapes of the hot kernels (0 in a split field = the built-in
 * default choice). */
typedef struct {
  int32_t h_lines;           /* h passes: grid lines (pencils) per workgroup of  */
                             /* three line passes, or -1: the z pass by pencils */
                             /* and x, y together on LDS z-slices               */
  int32_t damp_xy;           /* damped step: 1 = x and y transforms on LDS       */
                             /* z-slices (where they fit), 0 = line passes,     */
                             /* -1 = the default (slices up to 32^3)            */
  int32_t overlap_split[2];  /* split-K factor of the I/H product per species    */
  int32_t square_split[2];   /* split-K factor of the subspace products          */
  int32_t from_cache;        /* 1: every shape came from the cache file          */
  int32_t overlap_waves[2];  /* mixed: waves per 128 x 128 tile of the overlap   */
                             /* product, 8 (32 x 64 each) or 4 (64 x 64 each)  */
  int32_t combine_waves[2];  /* mixed: the same for the recombination product    */
} sky_tuning;

/* Autotuner.  Picks, for this box, the fastest of a few candidate launch
 * shapes of the dominant kernels: the pencils per workgroup of the h passes
 * or their LDS-slice variant, the slice or line variant of the damped step
 * (the FFT line kernels, keyed by grid size and precision), the split-K
 * factors of the overlap/Hamiltonian product and of the square subspace
 * products, and (mixed) the wave layout of the 128 x 128 output tiles of the
 * overlap and recombination plane products (keyed by state count, grid
 * points and precision).  Candidates
 * are timed with HIP events on the context's own buffers: call after
 * sky_init_box; the run overwrites h psi, phi and the subspace matrices (the
 * states are untouched).  Every candidate computes the same result up to
 * the order of floating-point sums.  cache_path (may be NULL): a flat JSON
 * object {"key": value}; shapes found there are used without timing, and
 * newly timed ones are merged into it.  For a mixed box the cache's FP64
 * entries for the same box (not timed here) are kept for the FP64 iterations
 * after a precision-ladder switch; without them those use the defaults.
 * out (may be NULL) receives the shapes in use.  Synchronises the stream.  Errors: SKY_ERR_INVALID (null
 * context, unwritable cache), SKY_ERR_HIP. */
int sky_autotune(sky_ctx* c, const char* cache_path, sky_tuning* out);

/* Launch shapes in use (defaults until sky_autotune). */
int sky_get_tuning(sky_ctx* c, sky_tuning* out);

/* HIP graphs (Fig. 1 iteration, launch side).  With graphs on, sky_iterate
 * captures the launch-only segments of an iteration once -- per species:
 * h psi, damped step, h phi, I and H (steps 2, 3a); psi = phi U (3e); and
 * the fields (4a, 4b, 5) -- and replays them; the host-driven subspace
 * solve (3b-3d) and the residual read-back run between replays.  Results
 * are those of the eager launches.  Graphs are dropped and recaptured when
 * the precision ladder switches or sky_autotune changes a launch shape;
 * phase timing (sky_set_timing) runs eagerly.  Needs a stream other than
 * the null stream.  Errors: SKY_ERR_INVALID, SKY_ERR_HIP. */
int sky_set_graphs(sky_ctx* c, int32_t enable);

/* Batched uneven boxes: iterates nbox independent contexts (any grid
 * sizes, state counts and precisions) until each one's Delta-eps <= tol
 * (tol <= 0: exactly max_iter iterations each).  Boxes are assigned to
 * nthreads host workers by longest-processing-time first on the cost of an
 * iteration (m^2 V for the products, m V log V for the FFT passes); each
 * worker owns a non-blocking HIP stream of default priority and runs its
 * boxes with graphs on, so up to nthreads boxes share the GPU at a time.
 * Every box stops at its own tolerance (per-box convergence mask).  reps[i]
 * and status[i] receive what sky_iterate returns for box i (SKY_OK or
 * SKY_NOT_CONVERGED, else an error code).  The contexts' own streams are
 * synchronised first and restored afterwards; a context may not appear
 * twice.  Returns SKY_OK, or the first box error (message names the box). */
int sky_batch_iterate(sky_ctx* const* ctxs, int32_t nbox, int32_t nthreads, int32_t max_iter,
                      double tol, sky_report* reps, int32_t* status);

/* The iteration of Fig. 1 with every decision on the device, replayed as
 * one HIP graph per iteration: chunk iterations are queued without any host
 * synchronisation, then the host reads the box's flags once.  On the
 * device: the Loewdin series' term count (Eq. Loewedin), the refinement's
 * stop test, Delta-eps (Eq. convergence) and the stop at
 * tol -- every kernel of the iteration reads the box's active flag first
 * and returns at once when it is cleared, so a converged box does no more
 * work (device-side convergence mask).  Where the host path would take
 * another branch (Cholesky far from orthonormality, the Jacobi fallback),
 * the device masks the rest of the iteration and the host finishes it on
 * the host path after the chunk (rep->eig_fallbacks counts these).  Results
 * equal sky_iterate's up to rounding: the series, refinement and residual
 * sums are the same arithmetic, and the refinement always forms the E^2
 * term.  The refinement takes at most desc.dev_refine_steps steps on the
 * device.  Contexts with options whose decisions stay on the host (learned
 * damping, the precision ladder, the paper-literal update, one_h, phase
 * timing, the null stream) run sky_iterate.  chunk >= 1.  Errors: as
 * sky_iterate. */
int sky_iterate_graph(sky_ctx* c, int32_t max_iter, double tol, int32_t chunk, sky_report* rep);

/* Batched uneven boxes with the device-decided iteration: the boxes are
 * assigned to nthreads workers as in sky_batch_iterate; each worker queues
 * a chunk of graph iterations for every unfinished box on its stream, then
 * drains the stream once and reads every box's flags (one host
 * synchronisation per worker per chunk, none per iteration).  reps[i] and
 * status[i] as sky_iterate_graph returns them.  Returns SKY_OK, or the
 * first box error (message names the box). */
int sky_batch_iterate_graph(sky_ctx* const* ctxs, int32_t nbox, int32_t nthreads,
                            int32_t max_iter, double tol, int32_t chunk, sky_report* reps,
                            int32_t* status);

/* Learned spectral preconditioner (an extension of Eq. dampstep, whose
 * damping x0 / (E0 + T_k) is fixed in the paper).  The learned step scales
 * the damping of state alpha in |k| shell s (8 equal |k| shells up to the
 * zone corner) by g = 4 sigmoid(MLP(|k_s| / |k|max, <h>_alpha / E0,
 * log10 share of the residual power in s, T(k_s) / E0)); the MLP is
 * 4-128-128-128-1, ReLU, BF16 weights, FP32 accumulation.
 *
 * sky_precond_collect: training rows from the current states of species q
 * (up to 32 sampled states x 8 shells): features, the target gains that
 * minimise the first-order residual |r - sum_s g_s (h - <h>) d_s|^2 of the
 * shell-restricted plain steps d_s, and the weights (residual share).
 * Overwrites h psi; *total = rows held (at most 16384; once the end is
 * reached, new rows overwrite the oldest from row 0).
 * sky_precond_train: Adam (lr) over all rows, weighted mean square error of
 * the gains; *loss = loss before the last update.
 * sky_precond_loss_grad: loss of the first nsamples rows and its gradient
 * (SKY_VIEW_PC_GRAD), parameters unchanged.
 * sky_precond_set_rows: declare the first nrows sample rows valid (rows
 * written by the caller through SKY_VIEW_PC_SAMPLES); 0 drops every row.
 * sky_precond_use: sky_iterate then takes the learned step; when the
 * residual Delta-eps after a learned step exceeds (1 + rise_tol) times the
 * one before it, the next 10 iterations use the plain damping (rise_tol = 0:
 * any rise; negative: never).  With retrain_every > 0, every retrain_every
 * iterations sky_iterate also collects rows from both species and takes 20
 * Adam steps (step size of the last sky_precond_train).  All synchronise
 * the stream.
 * Errors: SKY_ERR_INVALID (arguments, no rows, untrained network), SKY_ERR_HIP. */
int sky_precond_collect(sky_ctx* c, int32_t q, int32_t* total);
int sky_precond_train(sky_ctx* c, int32_t steps, double lr, double* loss);
int sky_precond_loss_grad(sky_ctx* c, int32_t nsamples, double* loss);
int sky_precond_set_rows(sky_ctx* c, int32_t nrows);
int sky_precond_use(sky_ctx* c, int32_t enable, double rise_tol, int32_t retrain_every);

/* Load a trained network into the learned damping: params_dev holds nparams
 * FP32 master parameters on the device (the layout of SKY_VIEW_PC_PARAMS;
 * nparams must equal that view's count), read only.  The BF16 copy used by
 * the kernels is rounded from them, the Adam moments are cleared and the
 * network counts as trained, so sky_precond_use may enable it at once (a
 * network trained on other boxes, carried to this one).
 * Errors: INVALID (count, null pointer). */
int sky_set_preconditioner(sky_ctx* c, const float* params_dev, int32_t nparams);

/* Wait for all work of the context's stream. */
int sky_sync(sky_ctx* c);

/* Description of the last failure on this host thread ("" if none). */
const char* sky_last_error(void);

/* Free host-side state of the context (not the caller's workspace). */
void sky_destroy(sky_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* SKY_H */
