/*
 * spec.h -- C ABI of the MI355X boundary oracle for spectrahedra and of the
 * random walks built on it (Chalkis, Emiris, Fisikopoulos, Repouskos,
 * Tsigaridas, "Efficient Sampling from Feasible Sets of SDPs and Volume
 * Approximation", arXiv:2010.03817).
 *
 * The problem (paper, Section 1, eq. (1)): a spectrahedron
 *     S = { x in R^n : F(x) = A0 + x_1 A1 + ... + x_n An  is PSD },
 * A_i symmetric, S bounded.  A line x + t v (or a degree-2 curve) meets the
 * boundary at the roots of det F(Phi(t)) nearest 0 (Lemma "PEP and S cap C");
 * the boundary normal there is (u^T A_i u)_i with u in ker F (Lemma
 * "Gradient of det F").
 *
 * Conventions shared by every entry point
 *  - Every call returns spec_status; SPEC_OK (0) on success.  Call-level
 *    errors (EINVAL, ENOMEM, EDEVICE) leave outputs unspecified.
 *  - Per-element outcomes go to an int32 status array (SPEC_OK,
 *    SPEC_NOT_INTERIOR, SPEC_UNBOUNDED, SPEC_NONSMOOTH, SPEC_NOCONV); values of
 *    NOT_INTERIOR elements are NaN.
 *  - Arrays are dense row-major float64 (batch x n) unless stated.
 *  - Entry points without a suffix take HOST pointers: inputs are read and
 *    outputs written during the call only; the call synchronises the device.
 *  - Entry points ending in _dev take DEVICE pointers and a hipStream_t passed
 *    as void* (NULL = the null stream); they are asynchronous on that stream.
 *    Buffers must stay live until the caller synchronises the stream.
 *  - A handle owns its device copies of the LMI and its scratch memory until
 *    spec_destroy; it is not thread-safe (use one stream per handle).
 *  - The library runs on the device current at spec_create; it never falls
 *    back to the CPU: without a usable device spec_create returns
 *    SPEC_EDEVICE.
 */
#ifndef SPEC_H
#define SPEC_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPEC_OK = 0,
    SPEC_EINVAL = 1,        /* bad argument (size < 1, NULL, non-symmetric block, ...) */
    SPEC_ENOMEM = 2,        /* device allocation failed */
    SPEC_EDEVICE = 3,       /* HIP runtime error or no device */
    SPEC_NOT_INTERIOR = 4,  /* start point not in the interior (Cholesky failed)   */
    SPEC_UNBOUNDED = 5,     /* t+ = +inf or t- = -inf along the curve              */
    SPEC_NONSMOOTH = 6,     /* hit at a point where the normal is not determined   */
    SPEC_REFLECT_CAP = 7,   /* more than rho reflections: the chain stayed         */
    SPEC_CERT_FALLBACK = 8, /* informational: learned bracket not certified        */
    SPEC_NOCONV = 9,        /* eigen iteration hit its cap; value is a bound        */
    SPEC_ENOTSUP = 10       /* size outside what the device kernels support        */
} spec_status;

typedef enum { SPEC_BLOCK_DENSE = 0, SPEC_BLOCK_DIAG = 1 } spec_block_kind;

typedef enum {
    SPEC_WALK_HNR = 0,      /* Hit-and-Run, Alg. Hit-and-Run                        */
    SPEC_WALK_CHNR = 1,     /* coordinate-directions Hit-and-Run                   */
    SPEC_WALK_BILLIARD = 2, /* billiard walk, Alg. Billiard                        */
    SPEC_WALK_HMC = 3       /* HMC with reflections, Alg. HMC_w_reflection         */
} spec_walk_kind;

typedef enum {
    SPEC_PREC_FP64 = 0,       /* FP64 pencil assembly                               */
    SPEC_PREC_FP32_ASM = 1,   /* FP32 MFMA assembly, FP32 accumulation              */
    SPEC_PREC_BF16X2_ASM = 2  /* bfloat16 hi+lo pairs on MFMA, FP32 accumulation    */
} spec_precision;

typedef struct spec_s* spec_handle;

/* Largest merged dense block the device kernels handle (one workgroup holds
 * the packed factor, m(m+1)/2 doubles, in the 160 KiB of LDS). */
#define SPEC_MAX_DENSE 200
/* Largest Krylov dimension accepted by spec_set_lanczos. */
#define SPEC_MAX_KRYLOV 160

/* Create a handle for the LMI F(x) = blkdiag_b (A_{b,0} + sum_i x_i A_{b,i}).
 *  n           number of coordinates (>= 1)
 *  nblocks     number of blocks (>= 1); block_size[b] >= 1, kind[b] as above
 *  A           host float64, blocks concatenated; DENSE block b: (n+1) full
 *              symmetric m_b x m_b row-major matrices A_{b,0}, ..., A_{b,n};
 *              DIAG block b: (n+1) vectors of length m_b (diagonals).
 * Dense blocks are merged into one block-diagonal dense block and diagonal
 * blocks into one diagonal block (the same LMI).  Returns SPEC_EINVAL if a
 * dense block is not symmetric to 1e-12 relative, SPEC_ENOTSUP if the merged
 * dense size exceeds SPEC_MAX_DENSE.  The handle owns device copies of A. */
spec_status spec_create(int n, int nblocks, const int* block_size, const int* kind,
                        const double* A, spec_handle* out);
spec_status spec_destroy(spec_handle h);

/* Settings of a handle.  Start from spec_options_default (zeroed fields are
 * not the defaults).
 *  precision     spec_precision of the pencil assembly (spec_set_precision)
 *  kmax, tol     Lanczos steps per cycle and residual tolerance
 *                (spec_set_lanczos; defaults 80 and 1e-8)
 *  refine_ratio  far-root refinement.  The rounding error of C = L^-1 B L^-T
 *                is about eps times its spectral radius rho, so from a start
 *                next to the boundary (rho = 1/|t-| large) the far root
 *                t+ = -1/lambda_min carries a relative error near
 *                eps rho / |lambda_min|.  When the run from x ends with
 *                rho > refine_ratio |lambda| for the eigenvalue of a root
 *                that decides the result, that root is recomputed from the
 *                shifted origin t0 = t1 (1 - 2^-10), t1 the first value: a
 *                Cholesky factor of F(x + t0 v) (certifying t0 inside) and a
 *                Lanczos run on which that root's eigenvalue dominates the
 *                spectrum (the pencil identity of Lemma "PEP and S cap C" with
 *                F(x) replaced by F(x + t0 v)).  Default 1e3; 0 disables.
 *  tol_loose     tolerance of the run from x on such a side: its value only
 *                places the origin of the refining run (default 1e-3).
 *  certify       1: after the oracle passes, every dense t+ of spec_intersect,
 *                spec_reflect and the line walks is checked by two Cholesky
 *                membership tests, F(x + t v) positive definite at
 *                t = t+ (1 - 1e-9) and not at t+ (1 + 1e-9) (two more
 *                factorisations per call); failures are flagged and counted.
 *                0 (default): the Kato-Temple interval of spec_certificates
 *                only.  Not applied to the uneven batch.
 *  escalate_ratio  precision split (spec_set_precision FP32 / BF16 hi+lo
 *                assembly): a call is redone with FP64 pencils when its
 *                reduced-precision F (F(p) of a curve) has min pivot / max
 *                pivot of its Cholesky factor below this (the pivots lie in
 *                [lambda_min, lambda_max], so lambda_min < ratio lambda_max
 *                then), when that F is not definite, and when the call ends at
 *                the boundary with a reflection to form (a reflection point
 *                pulled back by a relative 1e-6 needs the FP64 root); the
 *                factorisation and eigen solve are FP64 in every mode.
 *                Intersections without a reflection keep the reduced-precision
 *                roots.  Default 1e-3; 0 disables.  Counted as escalated.
 *  refresh_period  line walks (Hit-and-Run, coordinate Hit-and-Run, billiard)
 *                with FP64 pencils: F(x) is assembled from x in the first
 *                round of a spec_walk_run* call and every refresh_period rounds
 *                after it; in between a chain that moved by x <- x + s v is
 *                given F(x + s v) = F(x) + s B(v) (the identity of Lemma "PEP
 *                and S cap C"), so that those rounds assemble only B(v).  The
 *                sum adds one rounding of F per round, below the assembly's own
 *                (n + 1)-term rounding over a period.  A chain sent back to its
 *                step start (reflection cap, not-interior restart) skips its
 *                oracle calls until the next assembly round (not counted as
 *                calls).  Default 16; 1 assembles every round.
 * When the factor does not exist at t0 (t1 was too far out) the origin backs
 * off to t1 (1 - 2^-5) and then t1 / 2; only if those fail too is the plain
 * solve repeated at the full tolerance (counted as refine_failed in
 * spec_walk_stats, beside the refined calls). */
typedef struct {
    int precision;
    int kmax;
    double tol;
    double refine_ratio;
    double tol_loose;
    int certify;
    double escalate_ratio;
    int refresh_period;
} spec_options;

spec_status spec_options_default(spec_options* opt);
/* spec_create followed by spec_set_options (opt NULL: defaults); on an
 * options error the handle is destroyed and *out is NULL. */
spec_status spec_create_ex(int n, int nblocks, const int* block_size, const int* kind, const double* A,
                           const spec_options* opt, spec_handle* out);
spec_status spec_set_options(spec_handle h, const spec_options* opt);
spec_status spec_get_options(spec_handle h, spec_options* opt);

/* Sizes of a handle: n, merged dense size m, merged diagonal size md. */
spec_status spec_dims(spec_handle h, int* n, int* m, int* md);

const char* spec_status_str(spec_status s);

/* Lanczos settings of the extreme-eigenvalue step: at most kmax steps
 * (default 80) and the stopping test on the residual bound of the extreme
 * Ritz pairs, beta_{k+1} |s_k| <= max(tol |theta|, 100 eps rho) with rho the
 * spectral radius estimate (default tol 1e-8; the Ritz value error is then
 * about the square of the bound over the gap).  SPEC_ENOTSUP if the
 * tridiagonal would not fit in LDS for this handle's m. */
spec_status spec_set_lanczos(spec_handle h, int kmax, double tol);

/* Precision of the pencil assembly F(x), B(v) (and Q0, Q1, Q2 of curves):
 * SPEC_PREC_FP64 (default, FP64 MFMA), SPEC_PREC_FP32_ASM (coefficients and
 * the A-stack rounded to FP32, FP32 MFMA with FP32 accumulation),
 * SPEC_PREC_BF16X2_ASM (each FP32 operand split into a bfloat16 pair
 * hi + lo, products hi*hi + hi*lo + lo*hi on BF16 MFMA, FP32 accumulation).
 * The factorisation, the eigen solve and the reflection normal stay FP64;
 * the assembled pencils carry the reduced precision's rounding, so t+- move
 * by about that relative error times the conditioning of F(x). */
spec_status spec_set_precision(spec_handle h, int mode);

/* MEMBERSHIP (Alg. MEMBERSHIP, read as strict definiteness): interior[e] = 1
 * iff F(x_e) is positive definite (Cholesky succeeds). */
spec_status spec_membership(spec_handle h, int batch, const double* x, int8_t* interior);
spec_status spec_membership_dev(spec_handle h, int batch, const double* x, int8_t* interior,
                                void* stream);

/* INTERSECTION for lines (Alg. INTERSECTION with Phi(t) = x + t v):
 * t_minus <= 0 <= t_plus, the ends of the maximal interval around 0 where
 * F(x + t v) is PSD: t+ = -1/lambda_min(C), t- = -1/lambda_max(C),
 * C = L^{-1} B(v) L^{-T}, F(x) = L L^T, B(v) = sum v_i A_i; diagonal rows by
 * ratio.  status[e]: OK, NOT_INTERIOR (NaN outputs), UNBOUNDED (+-INFINITY),
 * NOCONV. */
spec_status spec_intersect(spec_handle h, int batch, const double* x, const double* v,
                           double* t_minus, double* t_plus, int32_t* status);
spec_status spec_intersect_dev(spec_handle h, int batch, const double* x, const double* v,
                               double* t_minus, double* t_plus, int32_t* status, void* stream);

/* Certified interval [t_lo, t_hi] of t+ for each element of the last
 * spec_intersect / spec_reflect call (and the last round of a walk) on this
 * handle, host arrays of `batch`.  A diagonal row's root is a ratio, exact up
 * to rounding: t_lo = t_hi = t+.  For the dense block, the run that fixes t+
 * from the origin t0 (0, the learned lower end or the refining origin) gives
 * the Ritz value theta >= lambda_min of C and its residual bound r; with the
 * second Ritz value bounded below by multisection on T_k, theta_2, the
 * Kato-Temple inequality places lambda_min in [theta - r^2 / (theta_2 -
 * theta), theta] (r enlarged by 8 eps times the spectral radius estimate for
 * the rounding of C), so t+ = t0 - 1/lambda_min lies in [t_lo, t_hi] with
 * t_hi the returned t+.  The interval is a posteriori: the gap uses the second
 * Ritz value, which bounds lambda_2 from above.  Elements whose interval is
 * wider than 2e-9 t+ are counted as uncertified (spec_walk_stats) and carry
 * bit 32 in spec_diag_call_flags; t_lo is -inf (no certified lower end) when
 * T_k shows no gap above theta (a second Ritz value at theta: a copy of the
 * converged one that a run continued past convergence grows) or the run did
 * not converge (SPEC_NOCONV); both NaN when there is no interval (no root was
 * computed: SPEC_NOT_INTERIOR, or membership only). */
spec_status spec_certificates(spec_handle h, int batch, double* t_lo, double* t_hi);

/* REFLECTION (Alg. REFLECTION, eq. (reflection)) for lines: t_plus as above,
 * s_out = v - 2 <v, w> w the reflected direction at x + t+ v, w_out (nullable)
 * the unit normal oriented outward (<v, w> >= 0).  A hit on a diagonal row
 * uses that row's gradient.  status[e]: as intersect, plus NONSMOOTH when the
 * smallest eigenvalue is numerically multiple or the normal vanishes (the
 * reflection is still returned).  If t+ = inf: s = v, w = 0, UNBOUNDED. */
spec_status spec_reflect(spec_handle h, int batch, const double* x, const double* v,
                         double* t_plus, double* s_out, double* w_out, int32_t* status);
spec_status spec_reflect_dev(spec_handle h, int batch, const double* x, const double* v,
                             double* t_plus, double* s_out, double* w_out, int32_t* status,
                             void* stream);

/* INTERSECTION for polynomial curves of degree 1 to SPEC_CURVE_MAX_DEGREE
 * (Alg. INTERSECTION, Lemma "PEP and S cap C", eq. (PEP)): with Q_k =
 * coef[e][k][0] A0 + sum_i coef[e][k][i] A_i (coef: batch x (degree+1) x
 * (n+1), row-major), the first positive / negative roots of
 * det(Q0 + t Q1 + .. + t^d Q_d) within |t| <= horizon
 * (+-INFINITY when there is none), i.e. the ends of the interval around 0 on
 * which Q(t) stays positive definite.  Q0 must be positive definite
 * (else NOT_INTERIOR, NaN outputs).  Dense blocks by certified Weyl steps:
 * each step factors Q(tau) and bounds lambda_min of L^-1 Q'(tau) L^-T and of
 * L^-1 Q2 L^-T from below (Lanczos Ritz value minus residual bound), so Q
 * stays definite over the step; diagonal rows by their scalar quadratics.
 * status[e]: OK, NOT_INTERIOR, NOCONV (the eigen solve of L^-1 Q'(tau) L^-T did
 * not converge; the bounds stay certified, the step only shorter).  Degree
 * >= 3: the same stepping with the Taylor coefficients of Q at tau,
 * L^-1 Q^(k)(tau) / k! L^-T, k = 1 .. d, each bounded from below by Lanczos,
 * and the step to the root of 1 + sum_k min(d_k, 0) s^k; diagonal rows by the
 * same stepping on their scalar polynomials; always FP64 pencils, and the
 * handle's workspace grows by (2 d + 3) rows per curve. */
#define SPEC_CURVE_MAX_DEGREE 6
spec_status spec_intersect_curve(spec_handle h, int batch, int degree, const double* coef, double horizon,
                                 double* t_minus, double* t_plus, int32_t* status);
spec_status spec_intersect_curve_dev(spec_handle h, int batch, int degree, const double* coef, double horizon,
                                     double* t_minus, double* t_plus, int32_t* status, void* stream);

/* Parameters of spec_walk_run (Section "Random walks").
 *  tau       billiard: step length ell = -tau ln(eta), eta ~ U(0,1) (Alg.
 *            Billiard; tau about the diameter); unused by Hit-and-Run
 *  rho       reflection cap per step; <= 0 means 10 n; a step with more than
 *            rho reflections leaves the chain where the step started
 *  gauss_a   Hit-and-Run target: exp(-gauss_a |x|^2) restricted to S
 *            (0 = uniform); the chord point is drawn from the target on the
 *            chord (Alg. Hit-and-Run)
 *  pullback  after a reflection the chain restarts from x + (1-pullback) t+ v
 *            (default 1e-6; the boundary point itself has a singular F)
 *  thin      store the point after every thin-th completed step (0 = none)
 *  max_rounds  stop after this many oracle rounds even if steps remain
 *            (<= 0: no limit); x_out then holds the last completed step
 *  resume    nonzero: continue the chains of the previous spec_walk_run_dev
 *            call on this handle (same kind, chains and seed) instead of
 *            starting from x0; `steps` then counts from the original start
 *  log_chains, log_cap, log_buf, log_count   optional device log of the
 *            segments of chains c < log_chains: records of 2n+4 doubles
 *            (x, v, t-, t+, chain, status) (HMC: (p, velocity, remaining travel time,
 *            first root u+ of the segment's pencil, chain, status)), log_count (device int32, zeroed
 *            by the caller) counts the records attempted.
 *  boltz_c, boltz_T   Boltzmann target exp(-<boltz_c, x> / boltz_T) restricted
 *            to S (the optimisation section, eq. (sdp)); boltz_c null = none,
 *            else n doubles (device memory for spec_walk_run_dev, host memory
 *            for spec_walk_run) and boltz_T > 0.  Hit-and-Run and coordinate
 *            Hit-and-Run draw the chord point from the truncated exponential
 *            exp(-t <c, v> / T); HMC follows p(t) = p + t v - t^2 c / (2T)
 *            (eq. (boltz_ode)), each segment one degree-2 curve whose horizon
 *            is the travel time left, and reflects the velocity v - t c / T at
 *            the hit.  Not with the billiard walk or with gauss_a > 0.
 *  ball_radius  billiard walk only: walk in S cap {|x| <= ball_radius} (the
 *            bodies S_i of eq. (mmc_vol)); a segment ends at the first of S's
 *            boundary, the sphere and the length left, and reflects on the
 *            sphere's radial normal when that comes first (0 = no ball; x0
 *            inside the ball). */
typedef struct {
    double tau;
    int rho;
    double gauss_a;
    double pullback;
    int thin;
    long long max_rounds;
    int resume;
    int log_chains;
    int log_cap;
    double* log_buf;
    int32_t* log_count;
    const double* boltz_c;
    double boltz_T;
    double ball_radius;
} spec_walk_params;

/* Totals over chains, counted over the rounds of this call (a resumed call
 * does not include the earlier calls' rounds): oracle calls, reflections, cap hits, not-interior
 * segments, nonsmooth reflections, completed steps, eigen non-convergence,
 * oracle rounds run, oracle calls whose learned bracket was not certified
 * (they fell back to the plain origin), oracle calls whose far root was
 * refined from a shifted origin (spec_options.refine_ratio), and refinements
 * whose factor at the shifted origin did not exist (the call then repeated the
 * plain solve at the full tolerance). */
typedef struct {
    double calls, reflections, cap_hits, not_interior, nonsmooth, steps, noconv, rounds, cert_fallback;
    double refined, refine_failed;
    double uncertified;  /* calls whose t+ interval (spec_certificates) is wider than 2e-9 t+ */
    double chol_cert_failed;  /* calls whose two-sided Cholesky certificate failed (spec_options.certify) */
    double escalated;    /* calls whose reduced-precision pencils were redone in FP64 (escalate_ratio) */
} spec_walk_stats;

/* Run `chains` independent chains of the walk `kind` from x0 (chains x n,
 * interior points) for `steps` steps each with seed `seed` (Philox4x32-10,
 * counter (chain, step, draw, tag)).  x_out (chains x n) receives the final
 * points; samples (nullable, chains x (steps/thin) x n) the thinned points;
 * stats (nullable, host) the totals.  Device pointers; asynchronous on
 * `stream` except that it reads a device flag every 16 rounds to stop when
 * all chains are done (and synchronises at the end when stats is given).
 * Kinds HNR, CHNR, BILLIARD, HMC (Alg. HMC with reflections for the Gaussian
 * target exp(-gauss_a |x|^2): travel time ell = tau eta, momentum N(0, I),
 * exact elliptic flow, each segment a degree-2 curve solved as in
 * spec_intersect_curve; or for the Boltzmann target of boltz_c, boltz_T;
 * exactly one of the two and tau > 0 required); SPEC_EINVAL for bad
 * arguments. */
spec_status spec_walk_run_dev(spec_handle h, int kind, int chains, const double* x0, long long steps,
                              uint64_t seed, const spec_walk_params* p, double* x_out, double* samples,
                              spec_walk_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Semidefinite optimisation by annealing (the optimisation section:
 * min <c, x> over S, eq. (sdp)).  Every chain walks the Boltzmann density
 * exp(-<c, x> / T_i) for walk_len steps at each temperature
 * T_i = T0 (1 - cool)^i, i = 0 .. iterations - 1, and keeps the best <c, x>
 * it has visited.  HMC (walk length one in the paper's runs) uses the travel
 * time scale tau_i = tau0 sqrt(T_i / T0): with time measured in units of
 * sqrt(T) this is HMC at temperature T with momenta N(0, T I) and a fixed
 * travel time, so the pull of c moves a chain by O(tau0^2 |c| / T0) per step
 * at every temperature.  Draws continue the chain's step counter across
 * temperatures (Philox counter (chain, step)).
 * ------------------------------------------------------------------------ */
typedef struct {
    int kind;        /* SPEC_WALK_HMC, SPEC_WALK_HNR or SPEC_WALK_CHNR */
    int iterations;  /* temperatures */
    int walk_len;    /* steps per temperature (>= 1) */
    double T0;       /* first temperature (> 0; the paper: about diam(S) for |c| = 1) */
    double cool;     /* T_{i+1} = T_i (1 - cool); <= 0: 1 / sqrt(n) */
    double tau0;     /* HMC travel-time scale at T0 (> 0 for HMC; the paper: the diameter) */
    int rho;         /* reflection cap per step (<= 0: 10 n) */
    double pullback; /* as spec_walk_params (<= 0: 1e-6) */
    double f_star;   /* known optimum for hit_iter (NaN: none) */
    double eps;      /* relative error that counts as reached (<= 0: 0.05) */
    int stop_when_reached;  /* nonzero (with f_star): stop after the first temperature at which
                               every chain is within eps; later entries of `best` repeat the last */
} spec_anneal_params;

/* Host arrays: x0 (chains x n) interior starts, c (n); outputs x_best
 * (chains x n, nullable), f_best (chains), best (chains x iterations,
 * nullable: each chain's best <c, x> after each temperature), hit_iter
 * (chains, nullable: first iteration whose best is within eps |f_star| of
 * f_star, -1 if none or f_star is NaN), stats (nullable: walk totals over all
 * temperatures).  Synchronises.  SPEC_EINVAL for bad arguments. */
spec_status spec_sdp_anneal(spec_handle h, const spec_anneal_params* p, int chains, const double* x0,
                            const double* c, uint64_t seed, double* x_best, double* f_best, double* best,
                            int32_t* hit_iter, spec_walk_stats* stats);

/* spec_walk_run_dev on HOST arrays (x0, x_out: chains x n; samples nullable:
 * chains x (steps/thin) x n), synchronous: the walk runs on the handle's
 * stream-less default queue and the outputs are copied back before return.
 * p->log_buf must be NULL (segment logs are device-side only). */
spec_status spec_walk_run(spec_handle h, int kind, int chains, const double* x0, long long steps, uint64_t seed,
                          const spec_walk_params* p, double* x_out, double* samples, spec_walk_stats* stats);

/* Save (restore = 0) or restore (restore = 1) the state of the chains of the
 * handle's last walk (points, step starts, directions, remaining lengths,
 * reflection and step counters, per-chain statistics) in device memory the
 * handle owns, so that a later resumed spec_walk_run_dev (same kind, chains
 * and seed) continues the same chains from the same state, e.g. under other
 * oracle settings.  Synchronises the device.  SPEC_EINVAL without a walk
 * state, or on restore when nothing was saved for the current state. */
spec_status spec_walk_state(spec_handle h, int restore);

/* ------------------------------------------------------------------------
 * Volume by Gaussian cooling (the Gaussian variant of multiphase Monte Carlo
 * that the paper's volume section names as an alternative to its ball
 * sequence): vol(S) = int_S f_0 * prod_i (int_S f_{i+1} / int_S f_i) with
 * f_i = exp(-a_i |x|^2), a_0 > ... > a_{phases-1} geometric, a_phases = 0.
 *  - int_S f_0 = (pi/a_0)^{n/2} Pr[X in S], X ~ N(0, I/(2 a_0)), from exact
 *    Gaussian draws and the membership oracle;
 *  - each ratio is the sample mean of exp((a_i - a_{i+1}) |x|^2) over points
 *    of Gaussian Hit-and-Run chains targeting f_i restricted to S (chains
 *    start from exact draws of f_0 inside S, are warm-started from the
 *    previous phase, and run burn_in steps after each change of target);
 *    the origin must be interior;
 *  - chains are split into `groups` independent groups; the estimate is the
 *    mean of the groups' log-volumes with a Student-t 95 % interval.
 * ------------------------------------------------------------------------ */
typedef struct {
    int phases;             /* cooling phases; <= 0: enough for a_{i+1} >= a_i (1 - 1/sqrt(n)), the
                               cooling rate under which each ratio has bounded relative variance
                               (at most 256; one count for a whole batch, the largest needed) */
    int samples_per_phase;  /* samples per phase over all chains; also exact draws per group for int f_0
                               (default 2000) */
    int chains;             /* chains, a multiple of groups (default 64) */
    int walk_len;           /* Hit-and-Run steps between recorded samples (default 10) */
    int groups;             /* independent groups for the interval (default 8) */
    double a0;              /* <= 0: chosen so that 50-90 % of N(0, I/(2 a0)) lies in S */
    double a_end;           /* <= 0: 1/(4 d^2), d the longest chord of a 64-chain Hit-and-Run pre-run */
    int burn_in;            /* Hit-and-Run steps at the start of each phase before samples are kept
                               (< 0: n, about one relaxation time of |x|^2 at rate 1/n per step; in a
                               batch the largest n, since all walks advance in lockstep) */
} spec_volume_params;

typedef struct {
    double a0, a_end;       /* the schedule's ends actually used */
    double p_inside;        /* fraction of the exact draws inside S */
    double oracle_calls;    /* line oracle calls of the walks */
    int phases;
    double log_terms[257];  /* [0] = log int f_0, [i] = log of ratio i (group means) */
} spec_volume_stats;

/* Estimate log vol(S); host outputs, asynchronous work on `stream`, synchronises.
 * EINVAL for bad parameters (phases <= 256, groups >= 2, chains % groups == 0). */
spec_status spec_volume_estimate(spec_handle h, const spec_volume_params* p, uint64_t seed, double* log_vol,
                                 double* ci_lo, double* ci_hi, spec_volume_stats* st, void* stream);

/* ------------------------------------------------------------------------
 * Volume by the ball sequence of eq. (mmc_vol): S_i = S cap rho_i B with
 * rho_0 = infinity.  In phase i the chains walk burn_in billiard steps in S_i
 * from where the last phase left them, then keep samples_per_chain points
 * walk_len steps apart.  The next radius rho_{i+1} is the q-quantile of |x|
 * over the first half of the samples (all chains); vol(S_{i+1}) / vol(S_i)
 * is the fraction of the second half inside rho_{i+1} B, per group of chains.
 * The sequence ends at the first ball with at least a fraction q inside S by
 * ball_draws exact uniform draws per group: vol(S_k) = vol(rho_k B) times the
 * group's fraction.  Chains outside the next ball move radially onto
 * (1 - 1e-6) rho_{i+1} (inside S, which is convex and holds 0).  0 must be an
 * interior point of S.  Phase i walks with the seed  seed + 7919 (i + 1).
 * ------------------------------------------------------------------------ */
typedef struct {
    int chains;             /* a multiple of groups (default 1024) */
    int groups;             /* independent groups for the interval (default 8) */
    int samples_per_chain;  /* per phase, even (default 16) */
    int walk_len;           /* billiard steps between kept points (default 1) */
    int burn_in;            /* steps at the start of each phase (< 0: n / 4; rounded up to walk_len) */
    double q;               /* target ratio of consecutive volumes (default 0.2) */
    int max_phases;         /* at most 256 (default 256) */
    int ball_draws;         /* exact draws per group for the stop test and the last ball (default 4096) */
    double tau;             /* billiard length scale (<= 0: 2 x the longest chord of a 64-chain Hit-and-Run
                               pre-run from 0) */
} spec_volume_balls_params;

typedef struct {
    int phases;             /* balls after S itself */
    double radii[257];      /* rho_1 .. rho_phases */
    double log_ratios[257]; /* [i] = mean over groups of log(vol(S_{i+1}) / vol(S_i)); [phases] = log vol(S_k) */
    double points;          /* billiard points generated (steps of all chains) */
    double oracle_calls;
    double tau;
} spec_volume_balls_stats;

/* log vol(S) and its 95 % interval over the groups (mean +- t_{0.975,g-1}
 * sd / sqrt(g)); host outputs, synchronises.  SPEC_EINVAL for bad parameters,
 * SPEC_NOCONV if max_phases balls do not reach one mostly inside S. */
spec_status spec_volume_balls(spec_handle h, const spec_volume_balls_params* p, uint64_t seed, double* log_vol,
                              double* ci_lo, double* ci_hi, spec_volume_balls_stats* st);

/* ------------------------------------------------------------------------
 * Uneven batching: many spectrahedra (different n and m) whose chains run
 * their oracle rounds together.  Each round assembles every instance's
 * pencils, then runs the per-chain oracle of all instances by a launch
 * strategy: 1 = one persistent launch whose workgroups take (instance, chain)
 * items, largest dense blocks first, from an atomic counter (LDS sized for
 * the largest m); 2 = one such launch per size class (m <= 64, m <= 128,
 * larger), so that small instances run many workgroups per compute unit;
 * 3 = one launch per instance.  0 = chosen by spec_batch_tune on first use.
 * With use_graph, a round is captured once per walk phase into a HIP graph
 * and replayed.  Batch calls need every handle in FP64 assembly
 * (SPEC_PREC_FP64; SPEC_ENOTSUP otherwise).
 * ------------------------------------------------------------------------ */
typedef struct spec_batch_s* spec_batch;

/* A batch over `count` handles; they stay owned by the caller and must
 * outlive the batch.  The batch has its own stream. */
spec_status spec_batch_create(int count, const spec_handle* hs, spec_batch* out);
spec_status spec_batch_destroy(spec_batch b);
spec_status spec_batch_set_strategy(spec_batch b, int strategy, int use_graph);
/* Time `rounds` uniform Hit-and-Run rounds of `chains` chains per instance
 * with each strategy (ms per round into ms_out[3], nullable) and keep the
 * fastest (*chosen, nullable).  The handles' walk state is overwritten. */
spec_status spec_batch_tune(spec_batch b, int chains, int rounds, double* ms_out, int* chosen);
/* One oracle round of the batch on given pairs (t- and t+ of every line, as
 * spec_intersect, Lemma "PEP and S cap C"): x and v are host arrays holding,
 * instance after instance, `chains` rows of that instance's n doubles
 * (row-major); t_minus, t_plus and status are host arrays of count * chains,
 * instance after instance.  The launch follows the batch's strategy (0 runs
 * strategy 1 without tuning).  The handles' walk state and call buffers are
 * overwritten.  Synchronises. */
spec_status spec_batch_intersect(spec_batch b, int chains, const double* x, const double* v, double* t_minus,
                                 double* t_plus, int32_t* status);
/* spec_volume_estimate for every instance, all walks advancing together:
 * log_vol, ci_lo, ci_hi: host arrays of `count`; oracle_calls (nullable):
 * total over instances.  Synchronises. */
spec_status spec_batch_volume(spec_batch b, const spec_volume_params* p, uint64_t seed, double* log_vol,
                              double* ci_lo, double* ci_hi, double* oracle_calls);

/* ------------------------------------------------------------------------
 * Learned boundary bracket.
 *
 * A small MLP maps (x, v) to predictions of (log t+, log(-t-)).  With a
 * network attached (spec_set_mlp) the billiard walk and spec_reflect start the
 * eigen solve from the shifted origin t_lo = exp(log t+_hat - delta) on the
 * line: when F(x + t_lo v) is positive definite (its Cholesky factor exists,
 * which certifies t_lo < t+), the same pencil identity as the plain path
 * (Lemma "PEP and S cap C", with F replaced by F(x + t_lo v)) gives
 * t+ = t_lo - 1/lambda_min(L_lo^-1 B L_lo^-T).  Near the boundary that
 * eigenvalue is far from the rest of the spectrum, so the Lanczos iteration
 * stops after a few steps.  Every Ritz value theta >= lambda_min, hence
 * t_lo - 1/theta >= t+ is a certified upper end of the bracket.  When the
 * Cholesky factor at t_lo does not exist the call redoes the factorisation at
 * the plain origin (status SPEC_CERT_FALLBACK, counted); results are the same
 * quantity as on the plain path in every case.
 *
 * Network: input [x, v] (2n, standardised), `hidden` layers of `width` with
 * exact GELU, output 2; FP32 master parameters, laid out per layer as W_l
 * (in x out, row-major) followed by b_l.  use_bf16 = 1 rounds weights and
 * activations to bfloat16 inside the products (BF16 MFMA, FP32 accumulation);
 * 0 computes in FP32 (FP32 MFMA).
 * ------------------------------------------------------------------------ */
typedef struct spec_mlp_s* spec_mlp;

typedef struct {
    int epochs;          /* passes over the training rows (default 20) */
    int batch;           /* minibatch rows (default 4096) */
    double lr;           /* Adam step size at the start (default 1e-3) */
    double lr_final;     /* step size at the end, cosine schedule (default 1e-5) */
    double val_frac;     /* last share of the rows held out for validation (default 0.1) */
    double quantile;     /* bracket half-width delta = this quantile of |log t+_hat - log t+|
                            on the validation rows (default 0.999) */
    uint64_t seed;       /* minibatch sampling */
    int keep_best;       /* nonzero: the loss on the validation rows is taken after every epoch and
                            the parameters of the best epoch are kept (early stopping) */
} spec_mlp_train_params;

typedef struct {
    double train_loss;   /* MSE on standardised targets, last epoch */
    double val_loss;     /* MSE on standardised targets, validation rows */
    double delta;        /* the bracket half-width at `quantile` */
    double err_median, err_p99, err_max;  /* |log t+_hat - log t+| on validation */
    double steps;        /* Adam steps taken */
    double val_rows;
    double err_q[8];     /* |log t+_hat - log t+| on validation at the levels
                            0.5, 0.7, 0.8, 0.9, 0.95, 0.99, 0.995, 0.999 */
    double val_loss_const; /* the same loss of the constant prediction (the training means) */
    double best_epoch;   /* keep_best: the epoch kept (1-based), else the last */
} spec_mlp_train_stats;

/* New network for n coordinates; parameters from Philox (key seed):
 * W ~ U(-1/sqrt(in), 1/sqrt(in)), b = 0.  width <= 1024, 1 <= hidden <= 8. */
spec_status spec_mlp_create(int n, int width, int hidden, int use_bf16, uint64_t seed, spec_mlp* out);
/* As spec_mlp_create; products = 1 appends two features computed from (x, v),
 * <x, v> and |x|^2, to the 2n inputs (2n + 2 inputs): the boundary distance
 * along v depends on them through a product of the inputs, which the network
 * does not learn from the raw coordinates on walk data. */
spec_status spec_mlp_create_ex(int n, int width, int hidden, int use_bf16, uint64_t seed, int products,
                               spec_mlp* out);
/* The feature standardisation of a trained network: mu and isd (inputs each:
 * features are (f - mu) * isd) and target = (mean, sd) of log t+ then of
 * log(-t-). */
spec_status spec_mlp_standardization(spec_mlp net, float* mu, float* isd, float* target);
spec_status spec_mlp_destroy(spec_mlp net);
spec_status spec_mlp_nparams(spec_mlp net, long long* np);
/* Copy the FP32 master parameters to / from host memory (np floats). */
spec_status spec_mlp_get_params(spec_mlp net, float* host);
spec_status spec_mlp_set_params(spec_mlp net, const float* host);
/* Raw network (no standardisation): Y (rows x 2) from X (rows x inputs: 2n, or 2n + 2 with products), device
 * pointers, float32. */
spec_status spec_mlp_forward_dev(spec_mlp net, int rows, const float* X, float* Y, void* stream);
/* Mean over rows x 2 entries of (Y - T)^2 and its gradient (np floats, device)
 * for the raw network; *loss is written on the host (the call synchronises). */
spec_status spec_mlp_loss_grad_dev(spec_mlp net, int rows, const float* X, const float* T, float* grad,
                                   double* loss, void* stream);
/* One Adam step (b1 0.9, b2 0.999, eps 1e-8) of the master parameters with a
 * device gradient; the step counter lives in the network. */
spec_status spec_mlp_adam_dev(spec_mlp net, const float* grad, double lr, void* stream);
/* Train on `rows` oracle results (x, v, t-, t+), device FP64 arrays (rows x n,
 * rows, rows): features and targets are standardised with statistics of the
 * training rows, minibatches are drawn uniformly with replacement.  Rows
 * must have finite t- < 0 < t+.  Synchronises; stats on the host. */
spec_status spec_mlp_train_dev(spec_mlp net, int rows, const double* x, const double* v, const double* t_minus,
                               const double* t_plus, const spec_mlp_train_params* p, spec_mlp_train_stats* st,
                               void* stream);
/* spec_mlp_train_dev on HOST arrays (x, v: rows x n; t_minus, t_plus: rows),
 * e.g. triples saved from earlier walks; the rows are copied to the device
 * for the call.  Synchronises. */
spec_status spec_mlp_train(spec_mlp net, int rows, const double* x, const double* v, const double* t_minus,
                           const double* t_plus, const spec_mlp_train_params* p, spec_mlp_train_stats* st);

/* Predictions log t+_hat and log(-t-_hat) (rows each, FP64, device) of the
 * trained (standardised) network. */
spec_status spec_mlp_predict_dev(spec_mlp net, int rows, const double* x, const double* v, double* log_tp,
                                 double* log_neg_tm, void* stream);
/* Attach a trained network to a handle (net NULL or mode 0 detaches).
 * mode 1: lower end certified by Cholesky, upper end by the Ritz value;
 * mode 2: additionally tests F(x + t_hi v), t_hi = exp(log t+_hat + delta),
 * and counts a definite F there as a fallback (informational).  The network
 * must stay alive while attached and have n equal to the handle's.  A run
 * from the network's shift tests convergence first at Lanczos step 6 (from
 * the plain origin: step 4). */
spec_status spec_set_mlp(spec_handle h, spec_mlp net, double delta, int mode);
/* Autotune the bracket half-width: for each of the ncand candidates, time the
 * learned reflection (mode 1) of `batch` device pairs (x, v) on `stream` with
 * HIP events (best of `reps` runs), write the milliseconds to ms_out (host,
 * ncand), and attach the network with the fastest candidate, returned in
 * *best (host).  Synchronises. */
spec_status spec_tune_mlp_delta_dev(spec_handle h, spec_mlp net, int batch, const double* x, const double* v,
                                    int ncand, const double* deltas, int reps, double* ms_out, double* best,
                                    void* stream);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * spec_intersect_noalloc_dev is spec_intersect_dev (same kernels, same
 * results) whose scratch memory (coefficient rows, assembled pencils, Lanczos
 * bases, per-chain first-pass results and the refinement queue) lives in one
 * static device array of SPEC_NOALLOC_SCRATCH_BYTES per device instead of the
 * handle's workspace: the call allocates nothing (the handle and its A-stack,
 * and the reduced-precision copy when spec_set_precision selected one, are
 * made beforehand).  Every call on a device shares that device's array, which
 * keeps the last call's contents (what must start at zero is cleared by a
 * kernel in each call), so calls that overlap on one device (other streams,
 * other threads, other handles) race.  The array needs, in bytes, about
 * bp (16 Kpad + 16 ldA + 8 kmax m + 64) for bp = batch rounded up to 64,
 * Kpad = round_up(n + 1, 16), ldA = round_up(m (m + 1) / 2 + md, 128), with
 * each piece rounded to 256 bytes (FP32/BF16 assembly adds 8 bp Kpad);
 * a larger batch returns SPEC_ENOTSUP before any work (n = m = 200, md = 400,
 * kmax 80: up to 128 pairs per call; n = m = 100: up to 384).  The per-call
 * diagnostics (spec_diag_lanczos_info, spec_diag_call_flags) do not see these
 * calls.
 * ------------------------------------------------------------------------ */
#define SPEC_NOALLOC_SCRATCH_BYTES (64u << 20)
spec_status spec_intersect_noalloc_dev(spec_handle h, int batch, const double* x, const double* v,
                                       double* t_minus, double* t_plus, int32_t* status, void* stream);

#ifdef __cplusplus
}
#endif
#endif
