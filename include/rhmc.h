/*
 * rhmc.h -- C ABI of the MI355X staggered-fermion solver library (librhmc.so).
 *
 * The library computes the hot path of two-flavour staggered RHMC as stated in
 * arXiv:1106.5673 ("QCD simulations with staggered fermions on GPUs"):
 *
 *   - the staggered hopping term D of Eq. (stag) with the phases
 *     eta_mu(n) = (-1)^(n_x + ... + n_{mu-1}) (Sec. 2), split into its
 *     even/odd blocks D_eo (odd -> even) and D_oe (even -> odd);
 *   - A = M^dagger M restricted to even sites, A = m^2 - D_eo D_oe
 *     (even/odd preconditioning, Sec. 2.1; M^dagger M of Eq. pseudofermions);
 *   - the shifted systems (A + sigma_i) x_i = b of Eq. (shifted), all solved
 *     from one Krylov space with a zero start (Sec. 4.3);
 *   - r(A) b = alpha0 b + sum_i alpha_i (A + beta_i)^-1 b, the rational
 *     approximation of the rooted power in Eq. (system_r) (Sec. 2.1).
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice  L = {Lx, Ly, Lz, Lt}, every extent even and >= 2; directions
 *          mu = 0..3 are x, y, z, t.  Site (x,y,z,t) has lexicographic index
 *          lex = x + Lx*(y + Ly*(z + Lz*t)), parity (x+y+z+t) mod 2 (0 = even)
 *          and, within its parity, index eo = lex / 2.  V = Lx*Ly*Lz*Lt,
 *          Vh = V/2.  Space is periodic; a hop across the time boundary is
 *          multiplied by t_bc (-1: antiperiodic).
 * Gauge    host complex128 [Lt][Lz][Ly][Lx][mu][row][col], (re, im)
 *          interleaved, each link in SU(3) (det = 1; the 12-real compressed
 *          copy reconstructs row 3 as conj(row1 x row2), Sec. 4.2).
 * Vectors  device colour vectors of one parity.  complex128 (double2) for
 *          RHMC_PREC_FP64: [nrhs][3][Vh], element (r, c, eo) at offset
 *          (r*3 + c)*Vh + eo.  complex64 (float2) for RHMC_PREC_FP32: one
 *          vector is [3][Vh] (offset c*Vh + eo); two or more are interleaved
 *          in pairs, pair q = (r = 2q, r = 2q + 1) being a [3][Vh] array of
 *          16-byte (re, im of 2q, re, im of 2q + 1) entries, so element
 *          (r, c, eo) is the complex64 at offset ((r/2)*3*Vh + c*Vh + eo)*2 +
 *          r%2 and a set of nrhs vectors occupies 2*ceil(nrhs/2)*3*Vh complex64
 *          (one 16-byte load then brings one colour of two vectors: the
 *          hopping kernel is bound by its number of loads).  With odd nrhs
 *          the second half of the last pair is read and overwritten with
 *          unspecified values.  Solver inputs and outputs are always
 *          complex128.
 * Streams  every call is enqueued on the caller's hipStream_t (0 = default
 *          stream).  rhmc_dslash_eo and rhmc_apply_mdagm are asynchronous;
 *          rhmc_multishift_cg and rhmc_rational_apply return after the
 *          solution and the statistics are complete.
 * Memory   the caller owns every vector and host array passed in; the library
 *          owns lattice and gauge objects, the packed links and a solver
 *          workspace cached inside the gauge object (allocated on first use
 *          for a given shape, freed by rhmc_gauge_destroy).
 * Errors   every call returns rhmc_status; on failure rhmc_last_error() gives
 *          a thread-local message.  Nothing aborts or throws across the ABI.
 */
#ifndef RHMC_H
#define RHMC_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RHMC_OK = 0,
    RHMC_ERR_INVALID_ARG = -1,   /* bad sizes, null pointers, odd extents, ... */
    RHMC_ERR_NONFINITE = -2,     /* a source or result holds NaN or Inf */
    RHMC_ERR_NOT_CONVERGED = -3, /* maxiter reached; outputs hold the last iterates */
    RHMC_ERR_HIP = -4,           /* a HIP runtime call failed */
    RHMC_ERR_OOM = -5,           /* device allocation failed */
    RHMC_ERR_UNSUPPORTED = -6    /* valid request this build does not implement */
} rhmc_status;

typedef enum { RHMC_PREC_FP64 = 0, RHMC_PREC_FP32 = 1 } rhmc_prec;

/* Link storage requested from rhmc_gauge_create (bit flags). */
#define RHMC_LINKS_FP64_18 1u /* 18 doubles per link: FP64 operator */
#define RHMC_LINKS_FP32_12 2u /* first two rows in FP32, third rebuilt: FP32 operator */
/* hi/lo split of Sec. 4.2: besides the FP32-12 copy (hi = RNE rounding of each
 * FP64 entry of rows 1-2) store lo = RNE rounding of (entry - hi).  Without
 * RHMC_LINKS_FP64_18 the FP64 operator (FP64 precision, reliable updates, true
 * residuals) is then built from hi + lo in FP64 arithmetic with the third row
 * rebuilt in FP64: about 48 significant bits per entry, relative operator error
 * ~2^-47 instead of ~2^-53, from 2 x 48 B per link instead of 144 B.  Implies
 * RHMC_LINKS_FP32_12. */
#define RHMC_LINKS_HILO_12 4u
/* FP64 rows 1-2 (12 doubles, 96 B per link), third row rebuilt in FP64 as
 * conj(row1 x row2): the storage of Sec. 4.2 in double precision.  The FP64
 * operator of choice when present (needs the links SU(3) to 1e-12). */
#define RHMC_LINKS_FP64_12 8u
/* All 18 reals in FP32 (72 B per link), no reconstruction: an FP32 operator
 * for links that are not SU(3).  Used when RHMC_LINKS_FP32_12 is absent. */
#define RHMC_LINKS_FP32_18 16u

typedef enum {
    RHMC_MODE_FP64 = 0,  /* every operator application and vector in FP64 */
    RHMC_MODE_MIXED = 1  /* FP32 operator and vectors, FP64 reliable updates */
} rhmc_mode;

typedef struct rhmc_lattice rhmc_lattice;
typedef struct rhmc_gauge rhmc_gauge;

typedef struct {
    double tol;             /* per-shift relative residual ||b-(A+s)x||/||b|| (default 1e-10) */
    int32_t maxiter;        /* Krylov iterations of the shared solve (default 100000) */
    int32_t mode;           /* rhmc_mode */
    int32_t reliable_every; /* MIXED: iterations between FP64 residual replacements (default 50) */
    int32_t refine;         /* nonzero: shifts whose FP64 true residual exceeds tol get a
                               warm-started CG on their own system (default 1) */
    int32_t block;          /* iterations between updates of the shifted solutions (1..50,
                               default 32).  MIXED replaces the residual at a block boundary
                               and so uses the divisor of reliable_every nearest to block
                               (between block/2 and 50; 25 for 50 and 32): replacements
                               fall exactly every reliable_every iterations.  Without such a
                               divisor block is kept and the cadence rounds up. */
    int32_t use_graph;      /* nonzero: replay each block of iterations as a hipGraph (default 1) */
    int32_t poll_every;     /* blocks launched between convergence polls (0 = automatic) */
    int32_t tune;           /* nonzero: time the Dslash launch shapes once and keep the best */
    int32_t per_shift;      /* nonzero: no shared Krylov space; every shifted system gets its
                               own CG from a zero start (batched up to 8 systems per launch,
                               sorted by shift, with reliable updates in MIXED mode), the
                               ordinary-solver alternative at the end of Sec. 4.3; stats then
                               give each system's own iterations, total_iterations is the
                               largest of them, refine_rounds counts this pass (default 0) */
    double fp64_head;       /* MIXED shared solve: iterate in FP64 until every right-hand side
                               has ||r|| <= fp64_head ||b||, then in FP32 with reliable updates.
                               A shifted solution cannot be restarted (Sec. 4.2), so FP32
                               rounding made while ||r|| is large stays in it; past the switch
                               it is scaled down by ||r||/||b||.  0 (default): min(1,
                               1e3 sqrt(tol)), i.e. 1e-2 at tol 1e-10 and no FP64 phase for
                               tol >= 1e-6; negative or >= 1: no FP64 phase; NaN is rejected */
    int32_t two_pass;       /* nonzero (FP64 mode, rational apply and pseudofermion action only):
                               a two-pass variant of the shared solve of Sec. 4.3 that the paper
                               does not describe.  Pass 1 runs the shared Krylov
                               solve with no shifted vectors and keeps each step's alpha and
                               beta; the weights w(k) with y = alpha0 b + sum_k w(k) r(k) follow
                               from them; pass 2 repeats the identical iteration (deterministic
                               reductions) and accumulates y from the residuals.  Twice the
                               operator work, no per-shift vectors.  stats->true_residual then
                               holds the recurrence residual |zeta_i| ||r|| / ||b|| of each shift
                               (no x_i is formed), and no refinement runs; maxiter is capped at
                               2^22 (24 B of recorded scalars per step and rhs).  UNSUPPORTED with
                               MIXED; INVALID_ARG with per_shift, rhmc_multishift_cg and the
                               force entry points (default 0) */
} rhmc_solver_params;

typedef struct {
    /* caller-owned arrays of nrhs*nshift entries, index r*nshift + i; each may be NULL */
    int32_t* iterations;     /* iteration at which shift i of rhs r met tol */
    double* true_residual;   /* final ||b - (A+sigma)x|| / ||b|| in FP64 */
    int32_t* refine_iterations;
    /* scalars filled by the library */
    int32_t total_iterations;   /* iterations of the shared Krylov solve */
    int32_t reliable_updates;
    int32_t refine_rounds;
    double time_ms;             /* host wall time of the call */
    double max_true_residual;
    int32_t fp64_head_iterations; /* MIXED: iterations of the shared solve run in FP64 */
    /* host wall time of each phase (ms, summed over groups of right-hand
     * sides; the phases end at host synchronisations, so they add up to the
     * solve part of time_ms) */
    double head_ms;     /* MIXED: the FP64 phase of the shared solve */
    double krylov_ms;   /* the shared solve after it (all of it in FP64 mode) */
    double check_ms;    /* FP64 true residuals of every shift, first check and rechecks */
    double refine_ms;   /* refinement solves of the shifts above tol */
} rhmc_solver_stats;

typedef struct {
    double alpha0;
    int32_t npole;
    const double* alpha; /* host [npole] */
    const double* beta;  /* host [npole], each > 0 (or >= 0 with m > 0) */
} rhmc_rational;

/* Fills the documented defaults. */
void rhmc_solver_params_default(rhmc_solver_params* p);

/* Lattice geometry (Sec. 2): L = {Lx, Ly, Lz, Lt}, each even and >= 2, V <= 2^26
 * (the kernels address a link plane of 4V entries with 32-bit byte offsets).
 * t_bc is +1 or -1.  *out must be released with rhmc_lattice_destroy. */
rhmc_status rhmc_lattice_create(const int32_t L[4], int32_t t_bc, rhmc_lattice** out);
void rhmc_lattice_destroy(rhmc_lattice* lat);

/* Neighbour table as the device kernels compute it: for every site of the given
 * parity, in eo order, the eo index of n+mu (columns 0..3) and n-mu (4..7).
 * out: host int32 [Vh][8].  sign (nullable): host int32 [Vh][8], the factor
 * eta_mu(n) * (boundary sign) that multiplies each hop.  Runs a kernel; blocks. */
rhmc_status rhmc_debug_neighbors(const rhmc_lattice* lat, int32_t parity, int32_t* out,
                                 int32_t* sign);

/* Upload and pack one gauge field (Sec. 4.2 storage: structure of arrays so that
 * consecutive sites read consecutive memory).  links: host array described
 * above, 4*V*9 complex128.  flags: any of RHMC_LINKS_*; 0 means FP32_12 plus
 * FP64_12, with FP64_18 instead of FP64_12 if row 3 of some link differs from
 * conj(row1 x row2) by more than 1e-12 and FP32_18 instead of FP32_12 if by
 * more than 1e-6.  The FP64 operator uses FP64_12 if stored, else FP64_18,
 * else hi + lo; the FP32 operator FP32_12 if stored, else FP32_18.  12-real
 * storage needs SU(3) links: INVALID_ARG if row 3 is off by more than 1e-12
 * (FP64_12) or 1e-6 (FP32_12), or links hold NaN/Inf.
 * The links are copied; the host array may be freed on return. */
rhmc_status rhmc_gauge_create(const rhmc_lattice* lat, const double* links, uint32_t flags,
                              hipStream_t stream, rhmc_gauge** out);
void rhmc_gauge_destroy(rhmc_gauge* g);

/* One application of the hopping term of Eq. (stag) between parities:
 * out_parity 0: out_even = D_eo in_odd;  1: out_odd = D_oe in_even.
 * prec FP64 uses the FP64 operator (FP64-12, FP64-18 or hi + lo links, see
 * rhmc_gauge_create) and complex128 vectors, FP32 the 12-real FP32 links and
 * complex64 vectors (paired when nrhs >= 2).  in and out: device vector sets
 * of nrhs vectors in the layout above, must not overlap.  1 <= nrhs <= 64. */
rhmc_status rhmc_dslash_eo(const rhmc_gauge* g, int32_t out_parity, rhmc_prec prec, int32_t nrhs,
                           const void* in, void* out, hipStream_t stream);

/* out = A in = m^2 in - D_eo D_oe in on even sites (Sec. 2.1).  Uses an odd-site
 * temporary from the gauge object's workspace.  Same layouts as rhmc_dslash_eo. */
rhmc_status rhmc_apply_mdagm(const rhmc_gauge* g, double m, rhmc_prec prec, int32_t nrhs,
                             const void* in, void* out, hipStream_t stream);

/* rhmc_apply_mdagm that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The odd-site temporary and the block partial sums
 * live in a static device array of 64 MiB that each GPU holds for the life of
 * the process; the call needs 8 * 8 * ceil(Vh/64) bytes (rounded up to 256)
 * plus one odd-parity vector set (nrhs * 3 * Vh * 16 bytes in FP64,
 * 2 * ceil(nrhs/2) * 3 * Vh * 8 in FP32 with nrhs >= 2) of it, and returns
 * RHMC_ERR_INVALID_ARG with nothing launched when that exceeds 64 MiB (e.g.
 * 48^3 x 12: up to 4 rhs in FP32, 2 in FP64).  All calls on one GPU share the
 * array, which keeps the last call's contents (nothing in it needs to start at
 * zero): calls that overlap on one GPU (other streams or host threads) race.
 * Same arguments, layouts, result bits and asynchrony as rhmc_apply_mdagm. */
rhmc_status rhmc_apply_mdagm_static(const rhmc_gauge* g, double m, rhmc_prec prec, int32_t nrhs,
                                    const void* in, void* out, hipStream_t stream);

/* Multi-shift CG (Sec. 4.3, Eq. shifted): x[r][i] = (A + shifts[i])^-1 b[r] for
 * every right-hand side r < nrhs and shift i < nshift, from the Krylov space of
 * the smallest shift with a zero starting guess.
 *   shifts: host [nshift], finite, >= 0, and > 0 if m == 0.  1 <= nshift <= 32.
 *   b:      device complex128 [nrhs][3][Vh];  x: device complex128 [nrhs][nshift][3][Vh].
 *   params: NULL for defaults.  stats: nullable.
 * Returns RHMC_ERR_NOT_CONVERGED (with x and stats holding the last state) when
 * some shift's FP64 true residual still exceeds tol. */
rhmc_status rhmc_multishift_cg(const rhmc_gauge* g, double m, int32_t nshift,
                               const double* shifts, int32_t nrhs, const void* b, void* x,
                               const rhmc_solver_params* params, rhmc_solver_stats* stats,
                               hipStream_t stream);

/* y[r] = alpha0 b[r] + sum_i alpha[i] (A + beta[i])^-1 b[r]  (Sec. 2.1, Eq. system_r).
 * b, y: device complex128 [nrhs][3][Vh] (may not overlap).  The shifted solutions
 * live in the gauge object's workspace.  stats as for rhmc_multishift_cg with
 * nshift = npole. */
rhmc_status rhmc_rational_apply(const rhmc_gauge* g, double m, const rhmc_rational* rat,
                                int32_t nrhs, const void* b, void* y,
                                const rhmc_solver_params* params, rhmc_solver_stats* stats,
                                hipStream_t stream);

/* Pseudofermion field of the Phi algorithm (Sec. 2.1) on even sites:
 *   phi_e = (M^dagger R)_e = m R_e - D_eo R_o      (M = m + D, D^dagger = -D),
 * whose covariance is A, i.e. phi is distributed as exp(-phi^dagger A^-1 phi)
 * for complex Gaussian R (real and imaginary parts N(0, 1/2)).  FP64 links.
 * r_even, r_odd, phi: device complex128 [nrhs][3][V/2] (R on the even and odd
 * sites, in the eo order of rhmc_dslash_eo); phi must not overlap R.
 * Asynchronous on `stream`.  For the rooted action below, the matching heat
 * bath is phi = r_h(A) R with r_h ~ x^{+1/8}: rhmc_rational_apply with that
 * approximation. */
rhmc_status rhmc_pf_phi(const rhmc_gauge* g, double m, int32_t nrhs, const void* r_even,
                        const void* r_odd, void* phi, hipStream_t stream);

/* Pseudofermion action S[r] = Re <phi_r, r(A) phi_r> for each right-hand side:
 * with r ~ x^{-1/4} this is the RHMC action of one pseudofermion carrying
 * det A^{1/4} (Eq. system_r with two flavours and two pseudofermions).  r(A)
 * phi is computed exactly as rhmc_rational_apply does (same params, same
 * stats, same per-shift FP64 certification); the inner products are FP64
 * with a fixed summation order.  phi: device complex128 [nrhs][3][V/2];
 * S: host double[nrhs].  Blocks until S is on the host.  On NOT_CONVERGED, S
 * holds the action of the last iterates. */
rhmc_status rhmc_pf_action(const rhmc_gauge* g, double m, const rhmc_rational* rat,
                           int32_t nrhs, const void* phi, double* S,
                           const rhmc_solver_params* params, rhmc_solver_stats* stats,
                           hipStream_t stream);

/* Pseudofermion force: the derivative of S = sum_r phi_r^dagger r(A) phi_r
 * with respect to the links, the molecular-dynamics force of Sec. 2.1.  For
 * the variation U_mu(n) -> exp(i eps T) U_mu(n) of one link (T Hermitian and
 * traceless), dS/deps = i Tr(T F_mu(n)) with
 *   F_mu(n) = TA(U_mu(n) M_mu(n)),   TA(X) = (X - X^dagger)/2 - Tr(X - X^dagger)/6,
 *   M_mu(n) = s_mu(n) sum_i alpha_i y_i(n+mu) x_i(n)^dagger   (n even),
 *            -s_mu(n) sum_i alpha_i x_i(n+mu) y_i(n)^dagger   (n odd),
 * x_i = (A + beta_i)^-1 phi (solved as rhmc_multishift_cg does, same params
 * and stats), y_i = D_oe x_i with the FP64 operator, s_mu(n) = eta_mu(n) times
 * the time-boundary sign of the hop n -> n+mu.  phi: device complex128
 * [nrhs][3][V/2]; force: device complex128 [Lt][Lz][Ly][Lx][4][3][3] (the
 * layout of the links given to rhmc_gauge_create), overwritten; traceless
 * anti-Hermitian.  Needs an FP64 operator.  Blocks until done. */
rhmc_status rhmc_pf_force(const rhmc_gauge* g, double m, const rhmc_rational* rat, int32_t nrhs,
                          const void* phi, void* force, const rhmc_solver_params* params,
                          rhmc_solver_stats* stats, hipStream_t stream);

/* Autotuner of the hopping kernel (the batching form's launch shapes): times
 * every launch variant (site processing order, hops per load batch, rows staged
 * in LDS per block) of one application D_oe on the given vectors
 * and keeps the fastest for this precision and rhs count in the gauge object
 * (the current variant stays unless another is more than 3% faster in the
 * final interleaved rounds); later calls of every entry point use it.  in: device vector set of nrhs
 * even-site vectors (layout above); out: the same, overwritten.  Blocks until
 * timed.
 * rhmc_multishift_cg and rhmc_rational_apply do the same when params->tune is set. */
rhmc_status rhmc_tune_dslash(rhmc_gauge* g, rhmc_prec prec, int32_t nrhs, const void* in,
                             void* out, hipStream_t stream);

/* The launch variant the hopping kernel currently uses for this precision and
 * rhs count (the measured default, or the autotuner's choice), for reports:
 * variant (host int32) = order + 8 * batch + 24 * shape + 96 * tile, with
 * order the site processing order 0..7 (0 even-odd index; 1..7 z-tiles of 1,
 * 2, 4, 6, 8, 3, 12 planes with t inside a tile, a tile that does not divide
 * Lz read as 1), batch the number of hops whose loads are issued together (1,
 * 2, 4 for 0..2), shape the block (0 256 sites; 1, 2 whole rows of an
 * xy-plane staged in LDS for the +-x and +-y hops, the fewest or the most
 * rows that fit whole waves of 64..512 sites and 48 KB of LDS, 256 sites
 * where none fits; 3 128 sites) and tile the right-hand sides per launch (0
 * all of them; 1 half of a class of four or eight, in two launches). */
rhmc_status rhmc_dslash_variant(const rhmc_gauge* g, rhmc_prec prec, int32_t nrhs,
                                int32_t* variant);

/* Pin the launch variant of the hopping kernel for this precision and rhs
 * count (0 <= variant < 192, layout as above).  Every variant computes the
 * same result bit for bit; they differ only in speed.  Marks the class as
 * tuned, so tune = 1 in later solver calls keeps it. */
rhmc_status rhmc_set_dslash_variant(rhmc_gauge* g, rhmc_prec prec, int32_t nrhs,
                                    int32_t variant);

/* ---------------------------------------------------------------- molecular dynamics
 * The update of Sec. 2.1 (Phi algorithm): momenta conjugate to the links,
 * Hamiltonian sum Tr(H^2) + S_g + S_f, a symmetric symplectic integrator and a
 * Metropolis test.
 *
 * Momenta: device double [8][4][2][V/2] = omega^a of link (mu, parity, eo),
 * H_mu(n) = sum_a omega^a T^a with T^a = lambda^a / 2 (Gell-Mann), so that
 * sum Tr(H^2) = (1/2) sum omega^2 and omega^a ~ N(0, 1) is the heat bath.
 * The caller draws them (and every other random number) and owns the array.
 *
 * Links evolve in place inside the gauge object: every storage it holds is
 * rewritten by each link update.  All of these entry points but
 * rhmc_kinetic need an FP64 link storage (FP64-12, FP64-18 or hi/lo) and
 * return RHMC_ERR_UNSUPPORTED without one.  Forces follow one convention: for U_mu(n) -> exp(i eps T)
 * U_mu(n), dS/deps = i Tr(T F_mu(n)), and a kick of size eps does
 * omega^a -= eps * i Tr(T^a F) (the flow that conserves the Hamiltonian with
 * dU/dtau = i H U). */

/* Plaquette (Wilson) action of Sec. 2,
 *   S_g = beta sum_n sum_{mu<nu} (1 - Re Tr P_{mu nu}(n) / 3),
 *   P_{mu nu}(n) = U_mu(n) U_nu(n+mu) U_mu(n+nu)^dagger U_nu(n)^dagger,
 * links periodic in every direction; FP64 sums in a fixed order.  S: host
 * double.  Blocks until S is on the host. */
rhmc_status rhmc_gauge_action(const rhmc_gauge* g, double beta, double* S, hipStream_t stream);

/* Gauge-force kick: mom -= eps * (i Tr(T^a F_g)) with
 *   F_g = -(beta/3) TA(U_mu(n) Sigma_mu(n)),
 *   Sigma_mu(n) = sum_{nu != mu} U_nu(n+mu) U_mu(n+nu)^dagger U_nu(n)^dagger
 *                              + U_nu(n+mu-nu)^dagger U_mu(n-nu)^dagger U_nu(n-nu),
 * the derivative of S_g.  mom: device, layout above, updated in place.
 * Asynchronous on `stream`. */
rhmc_status rhmc_gauge_force_kick(const rhmc_gauge* g, double beta, double eps, double* mom,
                                  hipStream_t stream);

/* Pseudofermion-force kick: mom -= eps * (i Tr(T^a F)) with F the force of
 * rhmc_pf_force for S = sum_r phi_r^dagger r(A) phi_r (same solves, params and
 * stats).  phi: device complex128 [npf][3][V/2].  Blocks until done. */
rhmc_status rhmc_pf_force_kick(const rhmc_gauge* g, double m, const rhmc_rational* rat,
                               int32_t npf, const void* phi, double eps, double* mom,
                               const rhmc_solver_params* params, rhmc_solver_stats* stats,
                               hipStream_t stream);

/* Link update U_mu(n) -> exp(i eps H_mu(n)) U_mu(n), followed by the FP64
 * reunitarisation of Sec. 4.1 (rows 1-2 Gram-Schmidt orthonormalised, row 3
 * the complex conjugate of their cross product), written to every storage of
 * g.  The exponential is the power series of the matrix scaled to norm 1/2,
 * squared back.  Asynchronous on `stream`. */
rhmc_status rhmc_update_links(rhmc_gauge* g, double eps, const double* mom, hipStream_t stream);

/* Kinetic term sum Tr(H^2) = (1/2) sum omega^2 (FP64, fixed order).  K: host
 * double.  Blocks until K is on the host. */
rhmc_status rhmc_kinetic(const rhmc_gauge* g, const double* mom, double* K, hipStream_t stream);

/* The current FP64 links of g in the layout of rhmc_gauge_create: device
 * complex128 [Lt][Lz][Ly][Lx][4][3][3] (caller-owned, overwritten; row 3
 * rebuilt where only rows 1-2 are stored).  Asynchronous on `stream`. */
rhmc_status rhmc_gauge_links(const rhmc_gauge* g, void* links, hipStream_t stream);

typedef struct {
    double beta;            /* gauge coupling of S_g */
    double mass;            /* quark mass m */
    double tau;             /* trajectory length (default 1) */
    int32_t n_md;           /* fermion steps per trajectory (default 12) */
    int32_t gauge_steps;    /* fermion step / gauge step, even >= 2 (default 10) */
    double lambda;          /* 2MN parameter, 0 <= lambda <= 1/2 (default 0.1931833275037836) */
    const rhmc_rational* force_rational;  /* r(x) of the fermion force (~x^{-1/4}) */
    rhmc_solver_params solver;            /* solves of the force (r_md, precision mode) */
} rhmc_md_params;

typedef struct {
    int32_t fermion_forces;   /* force evaluations (kicks merged where adjacent) */
    int32_t gauge_forces;
    int32_t link_updates;
    int64_t cg_iterations;    /* shared Krylov iterations summed over the force solves */
    double max_true_residual; /* worst certified residual of the force solves */
    double time_ms;
} rhmc_md_stats;

/* Defaults: beta 5.264, mass 0.01335, tau 1, n_md 12, gauge_steps 10, the
 * minimum-norm lambda, no rational, the solver defaults. */
void rhmc_md_params_default(rhmc_md_params* p);

/* Molecular dynamics over tau with the multi-step second-order minimum-norm
 * (2MN) scheme (Sec. 2.1).  One 2MN step of size h for a kick P and a drift Q:
 *   P(lambda h) Q(h/2) P((1 - 2 lambda) h) Q(h/2) P(lambda h).
 * The outer scheme (step delta = tau / n_md) kicks with the pseudofermion
 * force; each of its two drifts Q(delta/2) is made of gauge_steps/2 inner 2MN
 * steps of size delta / gauge_steps that kick with the gauge force and update
 * the links, so a trajectory makes n_md * gauge_steps gauge steps.  Kicks
 * between two link updates act on the same links and are summed into one
 * evaluation per force.  phi: device complex128 [npf][3][V/2]; mom: device
 * momenta (layout above), updated in place; links of g updated in place.
 * Blocks until done.  A force solve that misses its tolerance makes the call
 * return RHMC_ERR_NOT_CONVERGED after finishing the trajectory. */
rhmc_status rhmc_md_integrate(rhmc_gauge* g, const rhmc_md_params* params, int32_t npf,
                              const void* phi, double* mom, rhmc_md_stats* stats,
                              hipStream_t stream);

typedef struct {
    rhmc_md_params md;
    const rhmc_rational* heatbath_rational;  /* phi = r_hb(A) R (~x^{+1/8}) */
    const rhmc_rational* action_rational;    /* S_f = sum phi^dagger r_act(A) phi (~x^{-1/4}) */
    rhmc_solver_params metropolis_solver;    /* heat-bath and action solves (r_metro) */
} rhmc_hmc_params;

typedef struct {
    double kinetic[2];       /* before / after the molecular dynamics */
    double gauge_action[2];
    double pf_action[2];     /* summed over pseudofermions */
    double dH;               /* H(after) - H(before), summed part by part */
    int32_t accepted;
    rhmc_md_stats md;
    double time_ms;
} rhmc_trajectory_stats;

/* One trajectory of the Phi algorithm (Sec. 2.1): phi = r_hb(A) R, H before,
 * rhmc_md_integrate, H after, and the Metropolis test: accepted iff
 * u < exp(-dH).  On rejection, and on an error after the molecular dynamics
 * has started, the links of g are restored to their values at the start; mom
 * holds the final momenta either way.  R: device complex128
 * [npf][3][V/2], complex Gaussian (parts N(0, 1/2)); mom: device momenta drawn
 * N(0, 1) by the caller; u in [0, 1).  Blocks until done; stats required.  A
 * solve that misses its tolerance (heat bath, actions or forces) makes the
 * call return RHMC_ERR_NOT_CONVERGED after the trajectory is complete, with
 * the Metropolis decision taken on the values it produced. */
rhmc_status rhmc_trajectory(rhmc_gauge* g, const rhmc_hmc_params* params, int32_t npf,
                            const void* R, double* mom, double u, rhmc_trajectory_stats* stats,
                            hipStream_t stream);

const char* rhmc_status_string(rhmc_status s);
const char* rhmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RHMC_H */
