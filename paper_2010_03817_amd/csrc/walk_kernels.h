// Walk step machines (internal launch interface).
#pragma once
#include "spec_kernels.h"

namespace spec {

// Per-chain statistics: oracle calls, reflections, cap hits, not-interior,
// nonsmooth, completed steps, eigen non-convergence, learned-bracket fallbacks,
// far roots refined from a shifted origin, refinements whose factor failed,
// calls whose t+ interval was not certified to 2e-9, calls whose two-sided
// Cholesky certificate failed, calls redone in FP64 (precision escalation).
constexpr int WALK_NSTAT = 13;

struct WalkState {
    double* x;        // chains x n: current point
    double* xs;       // chains x n: point at the start of the current step
    double* v;        // chains x n: current direction
    double* ell;      // remaining length of the billiard step
    int32_t* nref;    // reflections in the current step
    long long* step;  // completed steps
    int32_t* active;  // 1 while the chain has steps left
    double* stats;    // chains x WALK_NSTAT
};

struct WalkArgs {
    int kind, chains, n;
    long long steps;
    uint64_t seed;
    double tau, gauss_a, pullback;
    int rho;
    const double* bc;  // Boltzmann target exp(-<bc, x> / bT) (nullable: none)
    double bT;
    double ball_r;     // billiard in S cap {|x| <= ball_r} (INFINITY: no ball)
    WalkState st;
    // oracle results of the current round
    const int32_t* status;
    const int32_t* flags;  // nullable: SPEC_FLAG_* bits of the oracle call
    const double* tm;
    const double* tp;
    const int32_t* hit;
    const double* wn;  // dense normal (chains x ldwn)
    int ldwn;
    const double* Astk;
    int ldA, P;
    // samples and logging
    double* samples;   // chains x nsamp x n (nullable): samples samp_first .. samp_first + nsamp - 1
    long long nsamp, samp_first;
    int thin;
    double* log_buf;   // log_cap records of (x, v, t-, t+, chain, status)
    int32_t* log_count;
    int log_cap, log_chains;
    // nullable (line walks that carry F(x) over between rounds): per chain the
    // move s of this round, x <- x + s v along the round's direction; NaN when
    // x is set otherwise (back to the step start), 0 when it stays
    double* upd_s;
};

hipError_t walk_init(const WalkArgs& a, const double* x0, hipStream_t s);
hipError_t walk_update(const WalkArgs& a, hipStream_t s);
// The update of `count` walks of `chains` chains each in one launch; dargs:
// their WalkArgs in device memory.
hipError_t walk_update_multi(const WalkArgs* dargs, int count, int chains, hipStream_t s);
hipError_t walk_finish(const WalkArgs& a, double* x_out, hipStream_t s);
hipError_t walk_count_active(int chains, const int32_t* active, int32_t* out, hipStream_t s);
hipError_t walk_sum_stats(int chains, const double* stats, double* out, hipStream_t s);
hipError_t walk_resume(const WalkArgs& a, hipStream_t s);
// HMC: coefficient rows of the segment's degree-2 pencil into Z and horizons.
hipError_t walk_hmc_prep(const WalkArgs& a, double* Z, int zrow0, int Kpad, double* horizon, hipStream_t s);
// Annealing: per-chain best <c, x> (init: from x0) and the history.
hipError_t anneal_track(int chains, int n, const double* x, const double* c, int it, int iters, double* xb,
                        double* fb, double* best, int32_t* hit, double f_star, double eps, bool init,
                        hipStream_t s);
// Ball-sequence volume: |x| of rows, exact uniform draws in rho B (point
// q = g * per_group + k from stream (g, k, tagbase | TAG_BALL*)), and chains
// moved radially into a ball of radius lim.
hipError_t row_norms(long long rows, int n, const double* X, double* out, hipStream_t s);
hipError_t ball_points(int count, int per_group, int n, uint64_t seed, uint32_t tagbase, double rho, double* X,
                       hipStream_t s);
hipError_t shrink_into_ball(int chains, int n, double* X, double lim, hipStream_t s);
// Volume helpers: exact Gaussian draws, per-group log-mean-exp of a phase,
// per-group membership counts.
hipError_t gauss_points(int count, int per_group, int n, uint64_t seed, double sd, double* X, hipStream_t s);
hipError_t phase_lse(int groups, int cpg, int nsamp, int n, const double* samples, double da, double* out,
                     hipStream_t s);
hipError_t count_groups(int groups, int per_group, const int8_t* flag, double* out, hipStream_t s);
// The first `chains` (<= 1024) draws inside S into out (chains x n); *found = how many there were.
hipError_t select_inside(int count, int n, const double* X, const int8_t* flag, int chains, double* out, int* found,
                         hipStream_t s);

}  // namespace spec
