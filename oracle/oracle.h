/*
 * oracle.h -- plain FP64 CPU reference of the spectrahedron boundary oracle
 * (Chalkis, Emiris, Fisikopoulos, Repouskos, Tsigaridas, "Efficient Sampling
 * from Feasible Sets of SDPs and Volume Approximation", arXiv:2010.03817).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
 * leg of the benchmark call this library to check the HIP path; the product
 * path never calls, links or loads it.  It shares no code with the HIP path.
 *
 * Conventions (identical in meaning to include/spec.h, written separately):
 *   - An LMI F(x) = A0 + sum_i x_i A_i (paper eq. (1)) is a list of blocks,
 *     F(x) = blkdiag_b F_b(x).  A DENSE block of size m stores (n+1) full
 *     symmetric m x m row-major matrices A_{b,0..n}; a DIAG block of size m
 *     stores (n+1) diagonals of length m.  Blocks are concatenated in A.
 *   - Per-element status codes match spec_status.
 */
#ifndef SPEC_ORACLE_H
#define SPEC_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 2, ORC_NOT_INTERIOR = 4,
       ORC_UNBOUNDED = 5, ORC_NONSMOOTH = 6, ORC_REFLECT_CAP = 7,
       ORC_NOCONV = 9 };
enum { ORC_DENSE = 0, ORC_DIAG = 1 };
enum { ORC_HNR = 0, ORC_CHNR = 1, ORC_BILLIARD = 2, ORC_HMC = 3 };

typedef struct orc_lmi orc_lmi;

int  orc_create(int n, int nblocks, const int* block_size, const int* kind,
                const double* A, orc_lmi** out);
void orc_destroy(orc_lmi* h);

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): out = bijection(ctr, key). */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Membership (Alg. MEMBERSHIP, read as a strict positive-definiteness test). */
int orc_membership(const orc_lmi* h, int batch, const double* x, int8_t* interior);

/* Intersection of the line x + t v with the boundary (Alg. INTERSECTION,
 * Lemma "PEP and S cap C"): t- <= 0 <= t+. */
int orc_intersect(const orc_lmi* h, int batch, const double* x, const double* v,
                  double* t_minus, double* t_plus, int32_t* status);

/* The same t- <= 0 <= t+ from membership alone: bisection on the convex
 * feasible interval {t : F(x + t v) > 0} with the Cholesky test of
 * orc_membership applied to F(x) + t B(v), down to adjacent doubles (the
 * definition of Lemma "PEP and S cap C"; no eigen solve, so the result does
 * not depend on the conditioning of F(x)).  guess (nullable, batch x 2:
 * t-, t+) only shortens the bracket search. */
int orc_line_bisect(const orc_lmi* h, int batch, const double* x, const double* v, const double* guess,
                    double* t_minus, double* t_plus, int32_t* status);

/* Reflection (Alg. REFLECTION, eq. (reflection), Lemma "Gradient of det F"):
 * t+, reflected direction s, unit outward normal w_hat (sign: <v,w> >= 0). */
int orc_reflect(const orc_lmi* h, int batch, const double* x, const double* v,
                double* t_plus, double* s_out, double* w_out, int32_t* status);

/* Degree-2 intersection: Q(t) = Q0 + t Q1 + t^2 Q2 with
 * Q_k = coef[k][0] A0 + sum_i coef[k][i+1] A_i, coef is batch x 3 x (n+1).
 * Returns the first positive / negative roots of det Q inside the horizon
 * (+-INFINITY when none). */
int orc_intersect_curve2(const orc_lmi* h, int batch, const double* coef, double horizon,
                         double* t_minus, double* t_plus, int32_t* status, int32_t* iters);

/* Random walks (Section "Random walks"). stats[0..7]: oracle calls,
 * reflections, cap hits, not-interior, nonsmooth, steps, no-convergence, 0. */
int orc_walk(const orc_lmi* h, int kind, int chains, const double* x0, int64_t steps,
             uint64_t seed, double tau, int rho, double gauss_a, double pullback,
             int thin, double* x_out, double* samples, double* stats);

/* Walks on the Boltzmann density exp(-<c, x> / T) truncated to S (kind
 * ORC_HNR, ORC_CHNR: truncated exponential on each chord; ORC_HMC: HMC with
 * reflections on p(t) = p + t v - t^2 c / (2T)); step k of chain j draws
 * with counter (j, step0 + k).  stats as orc_walk. */
int orc_walk_boltz(const orc_lmi* h, int kind, int chains, const double* x0, int64_t step0, int64_t steps,
                   uint64_t seed, double tau, int rho, const double* c, double T, double pullback,
                   int thin, double* x_out, double* samples, double* stats);

/* Annealing for min <c, x> over S: iteration i walks walk_len Boltzmann steps
 * at T_i = T0 (1 - cool)^i (HMC travel-time scale tau0 sqrt(T_i / T0)), then keeps
 * the best <c, x>; best (nullable) is chains x iters. */
int orc_sdp_anneal(const orc_lmi* h, int kind, int chains, const double* x0, const double* c, double T0,
                   double cool, int iters, int walk_len, uint64_t seed, double tau0, int rho, double pullback,
                   double* x_best, double* f_best, double* best);

/* One segment of the billiard walk for a given (x, v, ell): used to check the
 * device step machine on identical inputs. Writes x_new, v_new, ell_left and
 * flags[0] = 1 if reflected, flags[1] = status. */
int orc_billiard_segment(const orc_lmi* h, int batch, const double* x, const double* v,
                         const double* ell, double pullback, double* x_new, double* v_new,
                         double* ell_left, int32_t* flags);

/* Gaussian-cooling volume (telescoping product of integral ratios). */
int orc_volume(const orc_lmi* h, int phases, int samples_per_phase, int chains,
               int walk_len, uint64_t seed, double a0, double a_end, int n_groups,
               double* log_vol, double* ci_lo, double* ci_hi, double* log_ratios);

/* Volume by the ball sequence S_i = S cap rho_i B of eq. (mmc_vol): billiard
 * samples of each S_i, next radius the q-quantile of |x| (first half of the
 * samples), ratios from the second half per group, last ball when at least a
 * fraction q of it lies in S (ball_draws exact draws per group).  radii
 * (nullable, max_phases + 1) receives rho_0 = inf, rho_1, ...; ORC_NOCONV if
 * max_phases do not suffice.  0 must be interior to S. */
int orc_volume_balls(const orc_lmi* h, int chains, int spc, int walk_len, int burn_in, double q, int max_phases,
                     int ball_draws, uint64_t seed, double tau, int ng, double* log_vol, double* ci_lo,
                     double* ci_hi, double* radii, int* phases_out);

/* Small MLP: dims[0] -> ... -> dims[nl], GELU between layers, linear output.
 * params: for each layer l, W_l (dims[l] x dims[l+1], row-major) then b_l. */
int64_t orc_mlp_nparams(int nl, const int* dims);
int orc_mlp_forward(int nl, const int* dims, const double* params, int batch,
                    const double* X, double* Y);
/* loss = mean over batch*dims[nl] entries of (Y - T)^2; grad w.r.t. params. */
double orc_mlp_loss_grad(int nl, const int* dims, const double* params, int batch,
                         const double* X, const double* T, double* grad);
void orc_adam_step(int64_t np, double* params, const double* grad, double* m, double* v,
                   int step, double lr, double b1, double b2, double eps);

#ifdef __cplusplus
}
#endif
#endif
