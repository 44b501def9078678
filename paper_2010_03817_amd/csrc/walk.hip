// Step machines of the random walks (paper, Section "Random walks"): every
// round, every live chain runs one segment through the boundary oracle, and
// these kernels apply the walk's rule to the result.  A chain that finishes a
// step draws the next one at once, so every chain has a segment every round
// whatever its number of reflections (uneven work per step stays batched).
//
// Random numbers: Philox4x32-10 with key = seed and counter =
// (chain, step, draw, tag), the step being the chain's own count of
// completed steps.  Directions: Box-Muller normals normalised; billiard
// length ell = -tau ln(eta); chord position u (Hit-and-Run); coordinate
// floor(u n) (coordinate Hit-and-Run).
#include "common.h"
#include "walk_kernels.h"

namespace spec {

__device__ inline double dir_component(uint64_t seed, uint32_t chain, uint32_t step, uint32_t tag, int i) {
    double g0, g1;
    normal_pair(seed, chain, step, (uint32_t)(i >> 1), tag, g0, g1);
    return (i & 1) ? g1 : g0;
}

// Uniform direction on the sphere: normals 2d, 2d+1 of draw d, normalised.
// One wave per chain; each lane only writes its own coordinates.
__device__ inline void random_unit_dir(uint64_t seed, uint32_t chain, uint32_t step, uint32_t tag, int n,
                                       double* v, int lane) {
    double ss = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double g = dir_component(seed, chain, step, tag, i);
        ss += g * g;
    }
    ss = wave_sum(ss);
    const double inv = 1.0 / sqrt(ss);
    for (int i = lane; i < n; i += 64) v[i] = dir_component(seed, chain, step, tag, i) * inv;
}

// Begin step `step` of chain c: direction, and the billiard length.
__device__ inline void begin_step(const WalkArgs& a, int c, long long step64, int lane) {
    const WalkState& S = a.st;
    const uint32_t step = (uint32_t)step64;
    double* v = S.v + (size_t)c * a.n;
    if (a.kind == SPEC_WALK_CHNR) {
        double u0, u1;
        draw_u2(a.seed, (uint32_t)c, step, 0, TAG_COORD, u0, u1);
        int j = (int)floor(u0 * a.n);
        if (j >= a.n) j = a.n - 1;
        for (int i = lane; i < a.n; i += 64) v[i] = i == j ? 1.0 : 0.0;
    } else if (a.kind == SPEC_WALK_HMC) {
        // momentum v ~ N(0, I), not normalised (Alg. HMC with reflections)
        for (int i = lane; i < a.n; i += 64) v[i] = dir_component(a.seed, (uint32_t)c, step, TAG_MOM, i);
    } else {
        random_unit_dir(a.seed, (uint32_t)c, step, TAG_DIR, a.n, v, lane);
    }
    if (lane == 0) {
        if (a.kind == SPEC_WALK_BILLIARD) {
            double u0, u1;
            draw_u2(a.seed, (uint32_t)c, step, 0, TAG_LEN, u0, u1);
            S.ell[c] = -a.tau * log(u0);
        } else if (a.kind == SPEC_WALK_HMC) {
            double u0, u1;
            draw_u2(a.seed, (uint32_t)c, step, 0, TAG_LEN, u0, u1);
            S.ell[c] = a.tau * u0;  // travel time ell = tau eta, eta ~ U(0,1)
        } else {
            S.ell[c] = INFINITY;
        }
        S.nref[c] = 0;
    }
}

__global__ __launch_bounds__(256) void k_walk_init(WalkArgs a, const double* __restrict__ x0) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= a.chains) return;
    const WalkState& S = a.st;
    for (int i = lane; i < a.n; i += 64) {
        const double xi = x0[(size_t)c * a.n + i];
        S.x[(size_t)c * a.n + i] = xi;
        S.xs[(size_t)c * a.n + i] = xi;
    }
    if (lane == 0) {
        S.step[c] = 0;
        S.active[c] = a.steps > 0 ? 1 : 0;
        for (int k = 0; k < WALK_NSTAT; ++k) S.stats[(size_t)c * WALK_NSTAT + k] = 0.0;
    }
    if (a.steps > 0) begin_step(a, c, 0, lane);
}

// HMC-with-reflections trajectory for the Gaussian exp(-|x|^2 / (2 sigma^2)),
// sigma^2 = 1 / (2 gauss_a): the Hamiltonian flow is the ellipse
// Phi(theta) = p cos(theta) + sigma v sin(theta), theta = t / sigma, and with
// u = tan(theta / 2),  (1 + u^2) F(Phi) = F(p) + u 2 sigma B(v) + u^2 F(-p),
// a degree-2 pencil in u with the same roots.  A segment covers at most a
// quarter turn (u <= 1).  This kernel writes the pencil's coefficient rows
// [1, p], [0, 2 sigma v], [1, -p] and the horizon u_h = tan(theta_h / 2).
// For the Boltzmann target exp(-<c, x> / T) the trajectory is itself the
// degree-2 curve p + t v - t^2 c / (2T) (eq. (boltz_ode)) in t.
__global__ __launch_bounds__(256) void k_hmc_prep(WalkArgs a, double* __restrict__ Z, int zrow0, int Kpad,
                                                  double* __restrict__ horizon) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= a.chains) return;
    const WalkState& S = a.st;
    const int n = a.n;
    const double sigma = a.bc ? 0.0 : 1.0 / sqrt(2.0 * a.gauss_a);
    const double* x = S.x + (size_t)c * n;
    const double* v = S.v + (size_t)c * n;
    double* z0 = Z + (size_t)c * Kpad;
    double* z1 = Z + (size_t)(zrow0 + c) * Kpad;
    double* z2 = Z + (size_t)(2 * zrow0 + c) * Kpad;
    if (a.bc) {
        // Boltzmann trajectory p + t v - t^2 c / (2T): rows [1, p], [0, v],
        // [0, -c / (2T)] in t itself; the horizon is the travel time left
        const double h2 = -0.5 / a.bT;
        for (int k = lane; k < Kpad; k += 64) {
            const bool in = k >= 1 && k <= n;
            z0[k] = k == 0 ? 1.0 : (in ? x[k - 1] : 0.0);
            z1[k] = in ? v[k - 1] : 0.0;
            z2[k] = in ? h2 * a.bc[k - 1] : 0.0;
        }
        if (lane == 0) horizon[c] = fmax(S.ell[c], 0.0);
        return;
    }
    for (int k = lane; k < Kpad; k += 64) {
        double r0 = 0.0, r1 = 0.0, r2 = 0.0;
        if (k == 0) {
            r0 = 1.0;
            r2 = 1.0;
        } else if (k <= n) {
            r0 = x[k - 1];
            r1 = 2.0 * sigma * v[k - 1];
            r2 = -x[k - 1];
        }
        z0[k] = r0;
        z1[k] = r1;
        z2[k] = r2;
    }
    if (lane == 0) {
        const double half_pi = 1.5707963267948966;
        const double th = fmin(S.ell[c] / sigma, half_pi);
        horizon[c] = tan(0.5 * fmax(th, 0.0));
    }
}

// Continue chains that finished an earlier call's steps: a.steps is larger now.
__global__ __launch_bounds__(256) void k_walk_resume(WalkArgs a) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= a.chains) return;
    const WalkState& S = a.st;
    const long long k = S.step[c];
    if (S.active[c] || k >= a.steps) return;
    if (lane == 0) S.active[c] = 1;
    begin_step(a, c, k, lane);
}

// Exact draws from N(0, sd^2 I): point q = g * per_group + k uses normals
// 2d, 2d+1 of the stream (chain g, step k, tag TAG_GAUSS0).
__global__ void k_gauss_points(int count, int per_group, int n, uint64_t seed, double sd, double* __restrict__ X) {
    const int q = blockIdx.x;
    if (q >= count) return;
    const uint32_t g = (uint32_t)(q / per_group), k = (uint32_t)(q % per_group);
    for (int d = threadIdx.x; 2 * d < n; d += blockDim.x) {
        double g0, g1;
        normal_pair(seed, g, k, (uint32_t)d, TAG_GAUSS0, g0, g1);
        X[(size_t)q * n + 2 * d] = sd * g0;
        if (2 * d + 1 < n) X[(size_t)q * n + 2 * d + 1] = sd * g1;
    }
}

// Per group (block g): log of the mean of exp(da |x|^2) over the samples of
// the group's chains (chains [g cpg, (g+1) cpg), nsamp samples each), and the
// membership hit count of the exact draws of the group.
__global__ __launch_bounds__(256) void k_phase_lse(int cpg, int nsamp, int n, const double* __restrict__ samples,
                                                   double da, double* __restrict__ out) {
    __shared__ double red[8];
    const int g = blockIdx.x, t = threadIdx.x;
    const int cnt = cpg * nsamp;
    const double* base = samples + (size_t)g * cpg * nsamp * n;
    double mx = -INFINITY;
    for (int e = t; e < cnt; e += blockDim.x) {
        const double* x = base + (size_t)e * n;
        double r2 = 0.0;
        for (int i = 0; i < n; ++i) r2 += x[i] * x[i];
        mx = fmax(mx, da * r2);
    }
    mx = wave_max(mx);
    if ((t & 63) == 0) red[t >> 6] = mx;
    __syncthreads();
    mx = -INFINITY;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mx = fmax(mx, red[w]);
    __syncthreads();
    double sm = 0.0;
    for (int e = t; e < cnt; e += blockDim.x) {
        const double* x = base + (size_t)e * n;
        double r2 = 0.0;
        for (int i = 0; i < n; ++i) r2 += x[i] * x[i];
        sm += exp(da * r2 - mx);
    }
    sm = block_sum(sm, red);
    if (t == 0) out[g] = mx + log(sm) - log((double)cnt);
}

// Starting points: the first `chains` of the `count` draws that are inside S
// (flag set), in draw order; one workgroup, thread 0 selects.
__global__ void k_select_inside(int count, int n, const double* __restrict__ X, const int8_t* __restrict__ flag,
                                int chains, double* __restrict__ out, int* __restrict__ found) {
    __shared__ int pick[1024];
    __shared__ int np;
    if (threadIdx.x == 0) {
        int c = 0;
        for (int q = 0; q < count && c < chains && c < 1024; ++q)
            if (flag[q]) pick[c++] = q;
        np = c;
        *found = c;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < np * n; e += blockDim.x) out[e] = X[(size_t)pick[e / n] * n + e % n];
}

__global__ void k_count_groups(int groups, int per_group, const int8_t* __restrict__ flag, double* __restrict__ out) {
    const int g = blockIdx.x;
    if (g >= groups) return;
    int c = 0;
    for (int k = threadIdx.x; k < per_group; k += blockDim.x) c += flag[(size_t)g * per_group + k] != 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    __shared__ int red[16];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w];
        out[g] = (double)tot;
    }
}

// Truncated normal N(mu, sig^2) on [lo, hi] by inverting the CDF with u.
__device__ inline double trunc_normal_at(double mu, double sig, double lo, double hi, double u) {
    const double al = (lo - mu) / sig, be = (hi - mu) / sig;
    const double r2 = 1.4142135623730950488;
    double z;
    if (al >= 0.0) {  // upper tail: work with Q = 1 - Phi
        const double qa = 0.5 * erfc(al / r2), qb = 0.5 * erfc(be / r2);
        const double q = qa - u * (qa - qb);
        z = r2 * erfcinv(2.0 * q);
    } else if (be <= 0.0) {  // lower tail
        const double pa = 0.5 * erfc(-al / r2), pb = 0.5 * erfc(-be / r2);
        const double p = pa + u * (pb - pa);
        z = -r2 * erfcinv(2.0 * p);
    } else {
        const double pa = 0.5 * erfc(-al / r2), pb = 0.5 * erfc(-be / r2);
        const double p = pa + u * (pb - pa);
        z = p < 0.5 ? -r2 * erfcinv(2.0 * p) : r2 * erfcinv(2.0 * (1.0 - p));
    }
    double t = mu + sig * z;
    return fmin(fmax(t, lo), hi);
}

// Chord point of Hit-and-Run for exp(-<c, y> / T): along x + t v the density
// is exp(-lam t), lam = <c, v> / T, on [tm, tp]; inverse CDF from the end
// where the density is largest (lam >= 0: from tm with u; lam < 0: from tp
// with 1 - u, so t grows with u either way).
__device__ inline double trunc_exp_at(double lam, double tm, double tp, double u) {
    const double L = tp - tm;
    if (fabs(lam * L) < 1e-12) return tm + u * L;
    double t;
    if (lam > 0.0) {
        t = tm - log1p(u * expm1(-lam * L)) / lam;
    } else {
        const double mu = -lam;
        t = tp + log1p((1.0 - u) * expm1(-mu * L)) / mu;
    }
    return fmin(fmax(t, tm), tp);
}

// Finish a step: record the sample, advance the counter, start the next.
// Every lane of the chain's wave calls it; each lane touches its own
// coordinates only.
__device__ inline void end_step(const WalkArgs& a, int c, int lane) {
    const WalkState& S = a.st;
    const int n = a.n;
    for (int i = lane; i < n; i += 64) S.xs[(size_t)c * n + i] = S.x[(size_t)c * n + i];
    const long long k = S.step[c] + 1;
    if (a.samples && a.thin > 0 && k % a.thin == 0) {
        const long long j = k / a.thin - 1 - a.samp_first;
        if (j >= 0 && j < a.nsamp) {
            double* dst = a.samples + ((size_t)c * a.nsamp + j) * n;
            for (int i = lane; i < n; i += 64) dst[i] = S.x[(size_t)c * n + i];
        }
    }
    if (lane == 0) {
        S.step[c] = k;
        S.stats[(size_t)c * WALK_NSTAT + 5] += 1.0;
        if (k >= a.steps) S.active[c] = 0;
    }
    if (k < a.steps) begin_step(a, c, k, lane);
}

// The round's update of chain c by one wave (lane: its lane).
__device__ __forceinline__ void walk_update_chain(const WalkArgs& a, int c, int lane) {
    if (c >= a.chains) return;
    const WalkState& S = a.st;
    // the move of this round for a carried-over F(x) (see WalkArgs::upd_s)
    auto moved = [&](double sv) {
        if (a.upd_s && lane == 0) a.upd_s[c] = sv;
    };
    if (!S.active[c]) {
        moved(0.0);
        return;
    }
    const int32_t status = a.status[c];
    // no oracle call this round: the chain waits for a full assembly of F
    // (its move stays NaN); nothing is logged or counted
    if (status == WALK_STALE) return;
    const int n = a.n;
    double* x = S.x + (size_t)c * n;
    double* v = S.v + (size_t)c * n;
    double* st = S.stats + (size_t)c * WALK_NSTAT;
    const double tp = a.tp[c], tm = a.tm[c];
    // log the segment start (x, v) with its t-, t+
    if (a.log_buf && c < a.log_chains) {
        int slot = 0;
        if (lane == 0) slot = atomicAdd(a.log_count, 1);
        slot = __shfl(slot, 0, 64);
        if (slot < a.log_cap) {
            double* rec = a.log_buf + (size_t)slot * (2 * n + 4);
            for (int i = lane; i < n; i += 64) {
                rec[i] = x[i];
                rec[n + i] = v[i];
            }
            if (lane == 0) {
                // HMC segments log the remaining travel time in the t- slot
                rec[2 * n] = a.kind == SPEC_WALK_HMC ? S.ell[c] : tm;
                rec[2 * n + 1] = tp;
                rec[2 * n + 2] = (double)c;
                rec[2 * n + 3] = (double)status;
            }
        }
    }
    if (lane == 0) {
        st[0] += 1.0;
        if (status == SPEC_NOCONV) st[6] += 1.0;
        if (status == SPEC_CERT_FALLBACK) st[7] += 1.0;
        if (a.flags) {
            const int f = a.flags[c];
            if (f & SPEC_FLAG_REFINED) st[8] += 1.0;
            if (f & SPEC_FLAG_REFINE_FAILED) st[9] += 1.0;
            if (f & SPEC_FLAG_UNCERTIFIED) st[10] += 1.0;
            if (f & SPEC_FLAG_CHOL_CERT_FAILED) st[11] += 1.0;
            if (f & SPEC_FLAG_ESCALATED) st[12] += 1.0;
        }
    }
    if (status == SPEC_NOT_INTERIOR) {
        // cannot happen from an interior start; count it and restart the
        // step from its start point
        if (lane == 0) st[3] += 1.0;
        for (int i = lane; i < n; i += 64) x[i] = S.xs[(size_t)c * n + i];
        moved(NAN);
        end_step(a, c, lane);
        return;
    }
    if (a.kind == SPEC_WALK_HMC && a.bc) {
        // Boltzmann trajectory p + t v - t^2 c / (2T), velocity v - t c / T:
        // fly to the end of the travel time, or reflect at the first root
        const double iT = 1.0 / a.bT;
        const double ell = S.ell[c];
        const double ts = tp;
        if (!(ts <= ell) || !isfinite(ts)) {
            for (int i = lane; i < n; i += 64) {
                const double ci = a.bc[i];
                x[i] += ell * v[i] - 0.5 * ell * ell * ci * iT;
                v[i] -= ell * ci * iT;
            }
            if (lane == 0) S.ell[c] = 0.0;
            end_step(a, c, lane);
            return;
        }
        const int hit = a.hit[c];
        double nn = 0.0, vw = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double vh = v[i] - ts * a.bc[i] * iT;
            const double wi = hit == HIT_DENSE ? a.wn[(size_t)c * a.ldwn + i]
                                               : a.Astk[(size_t)(i + 1) * a.ldA + a.P + hit];
            nn += wi * wi;
            vw += wi * vh;
        }
        nn = wave_sum(nn);
        vw = wave_sum(vw);
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        const double coef = 2.0 * vw * inv * inv;
        const double t1 = (1.0 - a.pullback) * ts;
        for (int i = lane; i < n; i += 64) {
            const double ci = a.bc[i];
            const double wi = hit == HIT_DENSE ? a.wn[(size_t)c * a.ldwn + i]
                                               : a.Astk[(size_t)(i + 1) * a.ldA + a.P + hit];
            const double vh = v[i] - ts * ci * iT;
            x[i] += t1 * v[i] - 0.5 * t1 * t1 * ci * iT;
            v[i] = vh - coef * wi;
        }
        const int nref = S.nref[c] + 1;
        if (lane == 0) {
            if (!(nn > 0.0) || status == SPEC_NONSMOOTH) st[4] += 1.0;
            st[1] += 1.0;
            S.ell[c] = ell - ts;
            S.nref[c] = nref;
        }
        if (nref > a.rho) {
            if (lane == 0) st[2] += 1.0;
            for (int i = lane; i < n; i += 64) x[i] = S.xs[(size_t)c * n + i];
            end_step(a, c, lane);
        }
        return;
    }
    if (a.kind == SPEC_WALK_HMC) {
        // one segment of the trajectory: up to the boundary (reflect) or the
        // horizon (rotate), then continue while travel time is left
        const double sigma = 1.0 / sqrt(2.0 * a.gauss_a);
        const double half_pi = 1.5707963267948966;
        const double ell = S.ell[c];
        const double th_h = fmin(ell / sigma, half_pi);
        const double us = tp;
        double* xs_ = S.xs + (size_t)c * n;
        (void)xs_;
        if (!(us <= tan(0.5 * th_h)) || !isfinite(us)) {
            const double cs = cos(th_h), sn = sin(th_h);
            for (int i = lane; i < n; i += 64) {
                const double pi_ = x[i], vi = v[i];
                x[i] = pi_ * cs + sigma * vi * sn;
                v[i] = -pi_ / sigma * sn + vi * cs;
            }
            const double rest = ell - sigma * th_h;
            if (lane == 0) S.ell[c] = rest;
            if (!(rest > 1e-13 * sigma)) end_step(a, c, lane);
            return;
        }
        const double th = 2.0 * atan(us);
        const double cs = cos(th), sn = sin(th);
        // velocity at the hit point and the outward normal there
        const int hit = a.hit[c];
        double nn = 0.0, vw = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double vh = -x[i] / sigma * sn + v[i] * cs;
            const double wi = hit == HIT_DENSE ? a.wn[(size_t)c * a.ldwn + i]
                                               : a.Astk[(size_t)(i + 1) * a.ldA + a.P + hit];
            nn += wi * wi;
            vw += wi * vh;
        }
        nn = wave_sum(nn);
        vw = wave_sum(vw);
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        const double coef = 2.0 * vw * inv * inv;
        const double thp = (1.0 - a.pullback) * th;
        const double cp = cos(thp), sp = sin(thp);
        for (int i = lane; i < n; i += 64) {
            const double pi_ = x[i], vi = v[i];
            const double wi = hit == HIT_DENSE ? a.wn[(size_t)c * a.ldwn + i]
                                               : a.Astk[(size_t)(i + 1) * a.ldA + a.P + hit];
            const double vh = -pi_ / sigma * sn + vi * cs;
            x[i] = pi_ * cp + sigma * vi * sp;
            v[i] = vh - coef * wi;
        }
        const int nref = S.nref[c] + 1;
        if (lane == 0) {
            if (!(nn > 0.0) || status == SPEC_NONSMOOTH) st[4] += 1.0;
            st[1] += 1.0;
            S.ell[c] = ell - sigma * th;
            S.nref[c] = nref;
        }
        if (nref > a.rho) {
            if (lane == 0) st[2] += 1.0;
            for (int i = lane; i < n; i += 64) x[i] = S.xs[(size_t)c * n + i];
            end_step(a, c, lane);
        }
        return;
    }
    if (a.kind == SPEC_WALK_HNR || a.kind == SPEC_WALK_CHNR) {
        if (isfinite(tp) && isfinite(tm)) {
            double u0, u1;
            draw_u2(a.seed, (uint32_t)c, (uint32_t)S.step[c], 0, TAG_POS, u0, u1);
            double t;
            if (a.bc) {
                double cv = 0.0;
                for (int i = lane; i < n; i += 64) cv += a.bc[i] * v[i];
                cv = wave_sum(cv);
                // on the chord pulled back from both ends, as the oracle
                t = trunc_exp_at(cv / a.bT, (1.0 - a.pullback) * tm, (1.0 - a.pullback) * tp, u0);
            } else if (a.gauss_a > 0.0) {
                double xv = 0.0;
                for (int i = lane; i < n; i += 64) xv += x[i] * v[i];
                xv = wave_sum(xv);
                t = trunc_normal_at(-xv, 1.0 / sqrt(2.0 * a.gauss_a), tm, tp, u0);
            } else {
                t = tm + u0 * (tp - tm);
            }
            // every chord point at least the pull-back from the ends: a point
            // within the roots' own error of the boundary may lie outside
            t = fmin(fmax(t, (1.0 - a.pullback) * tm), (1.0 - a.pullback) * tp);
            for (int i = lane; i < n; i += 64) x[i] += t * v[i];
            moved(t);
        } else {
            moved(0.0);
        }
        end_step(a, c, lane);
        return;
    }
    // billiard (Alg. Billiard): move to the end of the segment or reflect
    const double ell = S.ell[c];
    double tlim = tp;  // nearest boundary along the segment (S, or S cap r B)
    if (a.ball_r < INFINITY) {
        // in S cap r B: the sphere's exit -<x, v> + sqrt(<x, v>^2 + r^2 - |x|^2)
        double xv = 0.0, xx = 0.0;
        for (int i = lane; i < n; i += 64) {
            xv += x[i] * v[i];
            xx += x[i] * x[i];
        }
        xv = wave_sum(xv);
        xx = wave_sum(xx);
        const double disc = xv * xv + a.ball_r * a.ball_r - xx;
        const double tb = -xv + sqrt(fmax(disc, 0.0));
        tlim = fmin(tp, tb);
        if (tb < tp && tb < ell) {
            // reflect on the radial normal w = x + tb v
            double ww = 0.0, wv = 0.0;
            for (int i = lane; i < n; i += 64) {
                const double wi = x[i] + tb * v[i];
                ww += wi * wi;
                wv += wi * v[i];
            }
            ww = wave_sum(ww);
            wv = wave_sum(wv);
            const double coef = ww > 0.0 ? 2.0 * wv / ww : 0.0;
            const double step_len = (1.0 - a.pullback) * tb;
            for (int i = lane; i < n; i += 64) {
                const double wi = x[i] + tb * v[i];
                x[i] += step_len * v[i];
                v[i] -= coef * wi;
            }
            moved(step_len);
            const int nref = S.nref[c] + 1;
            if (lane == 0) {
                st[1] += 1.0;
                S.ell[c] = ell - tb;
                S.nref[c] = nref;
            }
            if (nref > a.rho) {
                if (lane == 0) st[2] += 1.0;
                for (int i = lane; i < n; i += 64) x[i] = S.xs[(size_t)c * n + i];
                moved(NAN);
                end_step(a, c, lane);
            }
            return;
        }
    }
    if (!(tp < ell)) {
        // the step ends inside: at ell, but never nearer the boundary than the
        // pull-back of a reflection
        const double te = fmin(ell, (1.0 - a.pullback) * tlim);
        for (int i = lane; i < n; i += 64) x[i] += te * v[i];
        moved(te);
        end_step(a, c, lane);
        return;
    }
    // reflection: s = v - 2 <v, w> w with the outward unit normal w
    const int hit = a.hit[c];
    double nn = 0.0, vw = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double wi = hit == HIT_DENSE ? a.wn[(size_t)c * a.ldwn + i]
                                           : a.Astk[(size_t)(i + 1) * a.ldA + a.P + hit];
        nn += wi * wi;
        vw += wi * v[i];
    }
    nn = wave_sum(nn);
    vw = wave_sum(vw);
    const double step_len = (1.0 - a.pullback) * tp;
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    const double coef = 2.0 * vw * inv * inv;  // 2 <v, w_hat> / |w| along w
    for (int i = lane; i < n; i += 64) {
        const double wi = hit == HIT_DENSE ? a.wn[(size_t)c * a.ldwn + i]
                                           : a.Astk[(size_t)(i + 1) * a.ldA + a.P + hit];
        x[i] += step_len * v[i];
        v[i] -= coef * wi;
    }
    moved(step_len);
    const int nref = S.nref[c] + 1;
    if (lane == 0) {
        if (!(nn > 0.0) || status == SPEC_NONSMOOTH || (a.flags && (a.flags[c] & SPEC_FLAG_TIE))) st[4] += 1.0;
        st[1] += 1.0;
        S.ell[c] = ell - tp;
        S.nref[c] = nref;
    }
    if (nref > a.rho) {
        // too many reflections: the chain stays at the step's start point
        if (lane == 0) st[2] += 1.0;
        for (int i = lane; i < n; i += 64) x[i] = S.xs[(size_t)c * n + i];
        moved(NAN);
        end_step(a, c, lane);
    }
}

// One wave per chain.
__global__ __launch_bounds__(256) void k_walk_update(WalkArgs a) {
    walk_update_chain(a, blockIdx.x * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

// Every walk of a batch in one launch: bpi blocks of four chains per walk,
// walk k = blockIdx.x / bpi with its arguments in args[k] (device memory).
__global__ __launch_bounds__(256) void k_walk_update_multi(const WalkArgs* __restrict__ args, int bpi) {
    const WalkArgs& a = args[blockIdx.x / bpi];
    walk_update_chain(a, (blockIdx.x % bpi) * 4 + (threadIdx.x >> 6), threadIdx.x & 63);
}

__global__ void k_walk_finish(WalkArgs a, double* __restrict__ x_out) {
    const int c = blockIdx.x;
    if (c >= a.chains) return;
    for (int i = threadIdx.x; i < a.n; i += blockDim.x) x_out[(size_t)c * a.n + i] = a.st.xs[(size_t)c * a.n + i];
}

__global__ void k_count_active(int chains, const int32_t* __restrict__ active, int32_t* __restrict__ out) {
    __shared__ int red[1024];
    int s = 0;
    for (int c = threadIdx.x; c < chains; c += blockDim.x) s += active[c] != 0;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_sum_stats(int chains, const double* __restrict__ stats, double* __restrict__ out) {
    const int k = threadIdx.x;
    if (k >= WALK_NSTAT) return;
    double s = 0.0;
    for (int c = 0; c < chains; ++c) s += stats[(size_t)c * WALK_NSTAT + k];
    out[k] = s;
}

// Annealing bookkeeping, one wave per chain: f = <c, x>; a smaller f
// replaces the chain's best (value and point); best history and the first
// iteration within eps |f_star| of f_star.  init: the start point is the
// first best.
__global__ __launch_bounds__(256) void k_anneal_track(int chains, int n, const double* __restrict__ x,
                                                      const double* __restrict__ cv, int it, int iters,
                                                      double* __restrict__ xb, double* __restrict__ fb,
                                                      double* __restrict__ best, int32_t* __restrict__ hit,
                                                      double f_star, double eps, int init) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= chains) return;
    const double* xc = x + (size_t)c * n;
    double f = 0.0;
    for (int i = lane; i < n; i += 64) f += cv[i] * xc[i];
    f = wave_sum(f);
    const bool better = init || f < fb[c];
    if (better)
        for (int i = lane; i < n; i += 64) xb[(size_t)c * n + i] = xc[i];
    if (lane == 0) {
        const double b = better ? f : fb[c];
        fb[c] = b;
        if (init) {
            hit[c] = -1;
        } else {
            if (best) best[(size_t)c * iters + it] = b;
            if (hit[c] < 0 && isfinite(f_star) && b - f_star <= eps * fabs(f_star)) hit[c] = it;
        }
    }
}

__global__ __launch_bounds__(256) void k_row_norms(long long rows, int n, const double* __restrict__ X,
                                                   double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const long long r = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double xi = X[(size_t)r * n + i];
        s += xi * xi;
    }
    s = wave_sum(s);
    if (lane == 0) out[r] = sqrt(s);
}

// Uniform in rho B: direction g / |g| from normals of stream (grp, k,
// tagbase | TAG_BALL), radius rho u^(1/n) from (grp, k, tagbase | TAG_BALL_R).
// One wave per point.
__global__ __launch_bounds__(256) void k_ball_points(int count, int per_group, int n, uint64_t seed,
                                                     uint32_t tagbase, double rho, double* __restrict__ X) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= count) return;
    const uint32_t grp = (uint32_t)(q / per_group), k = (uint32_t)(q % per_group);
    double ss = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double g = dir_component(seed, grp, k, tagbase | TAG_BALL, i);
        ss += g * g;
    }
    ss = wave_sum(ss);
    double u0, u1;
    draw_u2(seed, grp, k, 0, tagbase | TAG_BALL_R, u0, u1);
    const double rad = rho * pow(u0, 1.0 / n) / sqrt(ss);
    for (int i = lane; i < n; i += 64) X[(size_t)q * n + i] = rad * dir_component(seed, grp, k, tagbase | TAG_BALL, i);
}

__global__ __launch_bounds__(256) void k_shrink_into_ball(int chains, int n, double* __restrict__ X, double lim) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= chains) return;
    double* x = X + (size_t)c * n;
    double s = 0.0;
    for (int i = lane; i < n; i += 64) s += x[i] * x[i];
    s = wave_sum(s);
    if (s > lim * lim) {
        const double sc = lim / sqrt(s);
        for (int i = lane; i < n; i += 64) x[i] *= sc;
    }
}

hipError_t row_norms(long long rows, int n, const double* X, double* out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_norms, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, rows, n, X, out);
    return hipGetLastError();
}

hipError_t ball_points(int count, int per_group, int n, uint64_t seed, uint32_t tagbase, double rho, double* X,
                       hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ball_points, dim3((count + 3) / 4), dim3(256), 0, s, count, per_group, n, seed, tagbase, rho,
                       X);
    return hipGetLastError();
}

hipError_t shrink_into_ball(int chains, int n, double* X, double lim, hipStream_t s) {
    if (chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_shrink_into_ball, dim3((chains + 3) / 4), dim3(256), 0, s, chains, n, X, lim);
    return hipGetLastError();
}

hipError_t anneal_track(int chains, int n, const double* x, const double* c, int it, int iters, double* xb,
                        double* fb, double* best, int32_t* hit, double f_star, double eps, bool init,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_anneal_track, dim3((chains + 3) / 4), dim3(256), 0, s, chains, n, x, c, it, iters, xb, fb,
                       best, hit, f_star, eps, init ? 1 : 0);
    return hipGetLastError();
}

hipError_t walk_init(const WalkArgs& a, const double* x0, hipStream_t s) {
    hipLaunchKernelGGL(k_walk_init, dim3((a.chains + 3) / 4), dim3(256), 0, s, a, x0);
    return hipGetLastError();
}
hipError_t walk_update(const WalkArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_walk_update, dim3((a.chains + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t walk_update_multi(const WalkArgs* dargs, int count, int chains, hipStream_t s) {
    if (count <= 0 || chains <= 0) return hipSuccess;
    const int bpi = (chains + 3) / 4;
    hipLaunchKernelGGL(k_walk_update_multi, dim3(count * bpi), dim3(256), 0, s, dargs, bpi);
    return hipGetLastError();
}
hipError_t walk_finish(const WalkArgs& a, double* x_out, hipStream_t s) {
    hipLaunchKernelGGL(k_walk_finish, dim3(a.chains), dim3(64), 0, s, a, x_out);
    return hipGetLastError();
}
hipError_t walk_count_active(int chains, const int32_t* active, int32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(1024), 0, s, chains, active, out);
    return hipGetLastError();
}
hipError_t walk_hmc_prep(const WalkArgs& a, double* Z, int zrow0, int Kpad, double* horizon, hipStream_t s) {
    hipLaunchKernelGGL(k_hmc_prep, dim3((a.chains + 3) / 4), dim3(256), 0, s, a, Z, zrow0, Kpad, horizon);
    return hipGetLastError();
}
hipError_t walk_resume(const WalkArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_walk_resume, dim3((a.chains + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t gauss_points(int count, int per_group, int n, uint64_t seed, double sd, double* X, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gauss_points, dim3(count), dim3(64), 0, s, count, per_group, n, seed, sd, X);
    return hipGetLastError();
}
hipError_t phase_lse(int groups, int cpg, int nsamp, int n, const double* samples, double da, double* out,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_phase_lse, dim3(groups), dim3(256), 0, s, cpg, nsamp, n, samples, da, out);
    return hipGetLastError();
}
hipError_t select_inside(int count, int n, const double* X, const int8_t* flag, int chains, double* out, int* found,
                         hipStream_t s) {
    if (chains > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_select_inside, dim3(1), dim3(256), 0, s, count, n, X, flag, chains, out, found);
    return hipGetLastError();
}
hipError_t count_groups(int groups, int per_group, const int8_t* flag, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_count_groups, dim3(groups), dim3(256), 0, s, groups, per_group, flag, out);
    return hipGetLastError();
}
hipError_t walk_sum_stats(int chains, const double* stats, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_stats, dim3(1), dim3(64), 0, s, chains, stats, out);
    return hipGetLastError();
}

}  // namespace spec
