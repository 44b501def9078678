// Fused per-chain line oracle (paper: Alg. INTERSECTION for Phi(t) = x + t v,
// Lemma "PEP and S cap C"; Alg. REFLECTION, Lemma "Gradient of det F").
//
// One workgroup per chain, 2m threads rounded up to whole waves.
//
//  1. F0 = F(x) + t0 B(v) (t0 = 0 on the plain path; the certified lower end of
//     the learned bracket otherwise) is read into LDS, packed by rows.
//  2. Blocked Cholesky F0 = L L^T and in-place triangular inverse W = L^{-1}
//     on 16x16 tiles with the FP64 matrix cores (v_mfma_f64_16x16x4f64);
//     the diagonal tiles are factored / inverted by one wave.
//  3. B(v) is held in registers: lane (r, h) keeps half h of the full
//     symmetric row r, so B a needs no cross-lane reduction.
//  4. Lanczos on C = W B W^T (W^T q from LDS, B a from registers, W b from
//     LDS) without reorthogonalisation; the basis goes to HBM for the Ritz
//     vector.  Every few steps the extreme Ritz values of T_k are bracketed by
//     multisection of Sturm counts and the residual bound beta_{k+1}|s_k| is
//     formed from the backward three-term recurrence of the eigenvector of
//     T_k; stop when it is below max(tol |theta|, 100 eps rho), rho the
//     spectral radius estimate (lambda_min only when asked).  The Ritz value
//     error is then about r^2 / gap.
//  5. With F(x + t v) = L (I + (t - t0) C) L^T:  t+ = t0 - 1/lambda_min,
//     t- = t0 - 1/lambda_max; diagonal rows by the ratio test; for a
//     reflection u = W^T z (z the Ritz vector of lambda_min) is a kernel
//     vector of F at the hit point and vec(u u^T) feeds the normal GEMM.
//
// Wave 0 steers the Lanczos iteration (Ritz values of T_k, stop test) and
// holds no part of B, so B's registers never meet the steering code.
// LDS at m = 200: 20100 doubles of the factor + 380 of scratch = 160 KiB.
#include "common.h"
#include "line_fused.h"

namespace spec {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int MAXH = 100;  // half-row length held in registers (m <= 200)

// Element (i, j) of tile (I, J) of the packed lower matrix; zero above the
// diagonal and outside m.
__device__ __forceinline__ double tl(const double* L, int m, int I, int J, int i, int j) {
    const int r = 16 * I + i, c = 16 * J + j;
    return (r < m && c <= r) ? L[pk(r, c)] : 0.0;
}

// acc += X * Y^T for 16x16 tiles X = (I1, J1), Y = (I2, J2) of L (sign sx on X).
__device__ __forceinline__ d4 mm_xyt(d4 acc, const double* L, int m, int I1, int J1, int I2, int J2, double sx,
                                    int lane) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double a = sx * tl(L, m, I1, J1, lane & 15, 4 * s + (lane >> 4));
        const double b = tl(L, m, I2, J2, lane & 15, 4 * s + (lane >> 4));
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Read a tile into the accumulator layout (lane l holds (l/16 + 4r, l%16)).
__device__ __forceinline__ d4 tile_to_acc(const double* L, int m, int I, int J, int lane) {
    d4 a;
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = tl(L, m, I, J, (lane >> 4) + 4 * r, lane & 15);
    return a;
}

// Write an accumulator tile back (lower part only on the diagonal).
__device__ __forceinline__ void acc_to_tile(double* L, int m, int I, int J, d4 a, int lane) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rr = 16 * I + (lane >> 4) + 4 * r, cc = 16 * J + (lane & 15);
        if (rr < m && cc <= rr) L[pk(rr, cc)] = a[r];
    }
}

// Unblocked Cholesky of diagonal tile K in place (one wave).  Rows past m act
// as identity.  Returns false if a pivot is not positive.
__device__ bool diag_chol(double* L, int m, int K, int lane) {
    bool ok = true;
    for (int j = 0; j < 16; ++j) {
        const int r = 16 * K + j;
        if (r >= m) break;
        const double d = L[pk(r, r)];
        if (!(d > 0.0)) { ok = false; break; }
        const double l = sqrt(d), inv = 1.0 / l;
        __builtin_amdgcn_wave_barrier();
        if (lane > j && lane < 16 && 16 * K + lane < m) L[pk(16 * K + lane, r)] *= inv;
        if (lane == 0) L[pk(r, r)] = l;
        __builtin_amdgcn_wave_barrier();
        // trailing update inside the tile: entries (i, k), j < k <= i < 16
        for (int e = lane; e < 256; e += 64) {
            const int i = e >> 4, k = e & 15;
            if (k > j && k <= i && 16 * K + i < m)
                L[pk(16 * K + i, 16 * K + k)] -= L[pk(16 * K + i, r)] * L[pk(16 * K + k, r)];
        }
        __builtin_amdgcn_wave_barrier();
    }
    return ok;
}

// D = inverse of the lower-triangular diagonal tile K (16 x 16, row-major in
// scratch D); rows past m are identity.  Lane c computes column c by forward
// substitution.  One wave.
__device__ void diag_inv(const double* L, int m, int K, double* D, int lane) {
    if (lane < 16) {
        const int c = lane;
        for (int i = 0; i < 16; ++i) {
            const int r = 16 * K + i;
            double val;
            if (i < c) {
                val = 0.0;
            } else if (r >= m) {
                val = i == c ? 1.0 : 0.0;
            } else {
                double s = i == c ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) s -= L[pk(r, 16 * K + k)] * D[k * 16 + c];
                val = s / L[pk(r, r)];
            }
            D[i * 16 + c] = val;
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Blocked Cholesky in LDS.  Returns false if F0 is not positive definite.
// `flag` is an LDS int; `D` 256 doubles of LDS scratch.
__device__ bool chol_blocked(double* L, int m, double* D, int* flag) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
    const int T = (m + 15) / 16;
    for (int K = 0; K < T; ++K) {
        if (wv == 0) {
            const bool ok = diag_chol(L, m, K, lane);
            if (lane == 0) *flag = ok ? 1 : 0;
            if (ok) diag_inv(L, m, K, D, lane);
        }
        __syncthreads();
        if (*flag == 0) return false;
        // panel: L_IK = A_IK D^T
        for (int I = K + 1 + wv; I < T; I += nw) {
            d4 acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double a = tl(L, m, I, K, lane & 15, 4 * s + (lane >> 4));
                const double b = D[(lane & 15) * 16 + 4 * s + (lane >> 4)];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
            acc_to_tile(L, m, I, K, acc, lane);
        }
        __syncthreads();
        // trailing update A_IJ -= L_IK L_JK^T, K < J <= I
        const int R = T - K - 1;
        for (int e = wv; e < R * (R + 1) / 2; e += nw) {
            int ii = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
            while (ii * (ii + 1) / 2 > e) --ii;
            const int jj = e - ii * (ii + 1) / 2;
            const int I = K + 1 + ii, J = K + 1 + jj;
            d4 acc = tile_to_acc(L, m, I, J, lane);
            acc = mm_xyt(acc, L, m, I, K, J, K, -1.0, lane);
            acc_to_tile(L, m, I, J, acc, lane);
        }
        __syncthreads();
    }
    return true;
}

// In-place triangular inverse W = L^{-1} of the packed lower factor: column
// blocks from the last one, W_IJ = -(sum_{K=J+1..I} W_IK L_KJ) L_JJ^{-1}.
__device__ void tri_inverse(double* L, int m, double* D) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
    const int T = (m + 15) / 16;
    for (int J = T - 1; J >= 0; --J) {
        if (wv == 0) diag_inv(L, m, J, D, lane);
        __syncthreads();
        // P_KJ = L_KJ D for K > J, in place
        for (int K = J + 1 + wv; K < T; K += nw) {
            d4 acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double a = tl(L, m, K, J, lane & 15, 4 * s + (lane >> 4));
                const double b = D[(4 * s + (lane >> 4)) * 16 + (lane & 15)];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
            acc_to_tile(L, m, K, J, acc, lane);
        }
        __syncthreads();
        // W_IJ = - sum_{K=J+1..I} W_IK P_KJ
        d4 res[4];
        int nres = 0;
        for (int I = J + 1 + wv; I < T; I += nw) {
            d4 acc{0.0, 0.0, 0.0, 0.0};
            for (int K = J + 1; K <= I; ++K) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double a = tl(L, m, I, K, lane & 15, 4 * s + (lane >> 4));
                    const double b = tl(L, m, K, J, 4 * s + (lane >> 4), lane & 15);
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
                }
            }
            res[nres++ & 3] = -acc;
        }
        __syncthreads();
        nres = 0;
        for (int I = J + 1 + wv; I < T; I += nw) acc_to_tile(L, m, I, J, res[nres++ & 3], lane);
        if (wv == 0) {
            for (int e = lane; e < 256; e += 64) {
                const int i = e >> 4, c = e & 15, r = 16 * J + i, cc = 16 * J + c;
                if (r < m && c <= i) L[pk(r, cc)] = D[e];
            }
        }
        __syncthreads();
    }
}

// Sturm count of the k x k tridiagonal (al, be) below x.
__device__ inline int sturm(const double* al, const double* be, int k, double x) {
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
        d = (al[i] - x) - (i ? be[i] * be[i] / d : 0.0);
        if (d == 0.0) d = -1e-300;
        cnt += d < 0.0;
    }
    return cnt;
}

// Extreme eigenvalue of T_k by multisection on one wave (65 points a round).
__device__ inline double extreme_ritz(const double* al, const double* be, int k, bool want_min) {
    const int lane = threadIdx.x & 63;
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < k; ++i) {
        const double rad = (i ? fabs(be[i]) : 0.0) + (i + 1 < k ? fabs(be[i + 1]) : 0.0);
        lo = fmin(lo, al[i] - rad);
        hi = fmax(hi, al[i] + rad);
    }
    const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
    lo -= pad;
    hi += pad;
    for (int it = 0; it < 12; ++it) {
        const double w = hi - lo;
        if (!(w > 2e-16 * fmax(fabs(lo), fabs(hi)))) break;
        const double x = lo + w * (double)(lane + 1) / 65.0;
        const int cnt = sturm(al, be, k, x);
        const unsigned long long mask = __ballot(want_min ? (cnt >= 1) : (cnt >= k));
        const int first = mask ? __ffsll((long long)mask) - 1 : 64;
        const double nlo = lo + w * (double)first / 65.0;
        const double nhi = first < 64 ? lo + w * (double)(first + 1) / 65.0 : hi;
        lo = nlo;
        hi = nhi;
    }
    return 0.5 * (lo + hi);
}

// Eigenvector of T_k for eigenvalue th by the backward recurrence from
// y_{k-1} = 1 (the Ritz vectors of converged extreme values decay towards
// the bottom, so this direction is the stable one).  Returns 1/|y| = |s_k|.
__device__ inline double backward_norm(const double* al, const double* be, int k, double th) {
    double y1 = 1.0, y0 = 0.0, ss = 1.0;  // y_{i}, y_{i+1}
    for (int i = k - 1; i >= 1; --i) {
        const double ym = ((th - al[i]) * y1 - (i + 1 < k ? be[i + 1] * y0 : 0.0)) / be[i];
        y0 = y1;
        y1 = ym;
        ss += ym * ym;
        if (ss > 1e280) {  // rescale
            const double sc = 1e-140;
            y0 *= sc;
            y1 *= sc;
            ss *= sc * sc;
        }
    }
    return 1.0 / sqrt(ss) * (ss > 0.0 ? 1.0 : 0.0);
}

__global__ __launch_bounds__(512) void k_line_fused(FusedArgs a) {
    extern __shared__ double lds[];
    const int m = a.m, P = a.P, md = a.md;
    const int chain = a.idx ? a.idx[blockIdx.x] : (int)blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
    double* L = lds;
    double* scr = lds + P;  // scratch; layout depends on the phase
    // factor phase: D tile [0, 256), flag at 256, diagonal-row reduction at 264..
    int* sflag = (int*)(scr + 256);
    double* rtp = scr + 264;
    double* rtm = rtp + 8;
    int* rj = (int*)(rtm + 8);
    int* rbad = rj + 8;

    const double* Fr = a.FB + (size_t)chain * a.ldfb;
    const double* Br = a.FB + (size_t)(a.brow0 + chain) * a.ldfb;
    const double t0 = a.shift ? a.shift[chain] : 0.0;
    int32_t st = SPEC_OK;

    // ---- diagonal rows: ratio test from x
    double dtp = INFINITY, dtm = -INFINITY;
    int dj = -1, bad = 0;
    for (int j = t; j < md; j += blockDim.x) {
        const double f = Fr[P + j], b = a.membership_only ? 0.0 : Br[P + j];
        if (!(f > 0.0)) bad = 1;
        const double r = b / f;
        if (r < 0.0) {
            const double tt = -1.0 / r;
            if (tt < dtp) { dtp = tt; dj = j; }
        } else if (r > 0.0) {
            dtm = fmax(dtm, -1.0 / r);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double otp = __shfl_xor(dtp, o, 64);
        const int oj = __shfl_xor(dj, o, 64);
        if (otp < dtp || (otp == dtp && oj >= 0 && (dj < 0 || oj < dj))) { dtp = otp; dj = oj; }
        dtm = fmax(dtm, __shfl_xor(dtm, o, 64));
        bad |= __shfl_xor(bad, o, 64);
    }
    if (lane == 0) { rtp[wv] = dtp; rtm[wv] = dtm; rj[wv] = dj; rbad[wv] = bad; }
    __syncthreads();
    dtp = INFINITY; dtm = -INFINITY; dj = -1; bad = 0;
    for (int w = 0; w < nw; ++w) {
        if (rtp[w] < dtp || (rtp[w] == dtp && rj[w] >= 0 && (dj < 0 || rj[w] < dj))) { dtp = rtp[w]; dj = rj[w]; }
        dtm = fmax(dtm, rtm[w]);
        bad |= rbad[w];
    }
    __syncthreads();
    double tp = dtp, tm = dtm;
    int hit = dj >= 0 ? dj : HIT_NONE;
    double lmin = 0.0, lmax = 0.0;
    int iters = 0;
    bool conv = true;
    int cert = 0;

    if (bad) st = SPEC_NOT_INTERIOR;
    if (!bad && m > 0) {
        // ---- upper certification of the learned bracket: F(x + t_hi v) must not be definite
        if (a.shift_hi) {
            const double th = a.shift_hi[chain];
            for (int e = t; e < P; e += blockDim.x) L[e] = Fr[e] + th * Br[e];
            __syncthreads();
            if (chol_blocked(L, m, scr, sflag)) cert = 2;
            __syncthreads();
        }
        // ---- factor F0 = F + t0 B
        for (int e = t; e < P; e += blockDim.x) L[e] = a.membership_only ? Fr[e] : Fr[e] + t0 * Br[e];
        __syncthreads();
        const bool ok = chol_blocked(L, m, scr, sflag);
        if (ok && !a.membership_only) tri_inverse(L, m, scr);
        if (!ok) {
            if (a.shift) cert = 1;
            else st = SPEC_NOT_INTERIOR;
        }
        if (ok && cert == 0 && !a.membership_only) {
            // Wave 0 steers (Ritz values, residual bounds, stop decision); waves
            // 1.. hold B and run the matrix-vector products.  Both run the same
            // sequence of barriers.
            const int hm = (m + 1) >> 1;
            const int tw = t - 64;
            const int r = tw >> 1, h = tw & 1;
            const bool worker = wv >= 1;
            const bool own = worker && r < m;
            const int c0 = h * hm;
            const int kmax = a.kmax;
            double* slot = scr;            // 2 MAXH (zero past m)
            double* al = scr + 2 * MAXH;   // kmax
            double* be = al + kmax;        // kmax + 1
            double* red = be + kmax + 1;   // 8
            double* sres = red + 8;        // 8: theta_min, r_min, theta_max, r_max, stop, k
            double* Qg = a.Q + (size_t)chain * a.ldq;
            for (int e = m + t; e < 2 * MAXH; e += blockDim.x) slot[e] = 0.0;
            const int R0w = 32 * (wv - 1);  // first column of this worker wave in W^T x
            // start vector (deterministic, positive)
            double qr = 0.0;
            if (own) {
                u4 hsh = philox10(u4{(uint32_t)r, 0x5eedu, 0u, 0x51a7u}, 0x2010u, 0x3817u);
                qr = 0.5 + (double)(hsh.x >> 11) * (1.0 / 2097152.0);
            }
            double nq = block_sum((own && h == 0) ? qr * qr : 0.0, red);
            qr *= 1.0 / sqrt(nq);
            if (worker) {
                double breg[MAXH];
#pragma unroll
                for (int k = 0; k < MAXH; ++k) {
                    const int c = c0 + k;
                    double v = 0.0;
                    if (own && k < hm && c < m) v = c <= r ? Br[pk(r, c)] : Br[pk(c, r)];
                    breg[k] = v;
                }
                double qprev = 0.0, bprev = 0.0;
                for (int j = 0; j < kmax; ++j) {
                    if (own && h == 0) {
                        Qg[(size_t)j * m + r] = qr;
                        slot[r] = qr;
                    }
                    __syncthreads();  // B1
                    // a = W^T q, lanes (c, h) over row halves of the wave's band
                    double av = 0.0;
                    if (own) {
                        const int c = r, mid = (R0w + m) >> 1;
                        const int rb = h == 0 ? R0w : mid, re = h == 0 ? mid : m;
                        for (int rr = rb; rr < re; ++rr)
                            if (rr >= c) av += L[pk(rr, c)] * slot[rr];
                    }
                    av += __shfl_xor(av, 1, 64);
                    __syncthreads();  // B2
                    if (own && h == 0) slot[r] = av;
                    __syncthreads();  // B3
                    // b = B a from registers
                    double bv = 0.0;
                    {
                        const double* sv = slot + c0;
#pragma unroll
                        for (int kk = 0; kk < MAXH; kk += 4) {
                            bv += breg[kk] * sv[kk];
                            bv += breg[kk + 1] * sv[kk + 1];
                            bv += breg[kk + 2] * sv[kk + 2];
                            bv += breg[kk + 3] * sv[kk + 3];
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                    bv += __shfl_xor(bv, 1, 64);
                    __syncthreads();  // B4
                    if (own && h == 0) slot[r] = bv;
                    __syncthreads();  // B5
                    // c = W b
                    double cv = 0.0;
                    if (own) {
                        const int half = (r + 2) >> 1;
                        const int kb = h == 0 ? 0 : half, ke = h == 0 ? half : r + 1;
                        const double* row = L + pk(r, 0);
                        for (int kk = kb; kk < ke; ++kk) cv += row[kk] * slot[kk];
                    }
                    cv += __shfl_xor(cv, 1, 64);
                    const double alj = block_sum((own && h == 0) ? qr * cv : 0.0, red);  // B6, B7
                    cv -= alj * qr + bprev * qprev;
                    const double bn = sqrt(block_sum((own && h == 0) ? cv * cv : 0.0, red));  // B8, B9
                    __syncthreads();  // B10 (control wave stores alpha, beta)
                    __syncthreads();  // B11 (control wave decides)
                    if (sres[4] != 0.0) break;
                    qprev = qr;
                    qr = cv * (1.0 / bn);
                    bprev = bn;
                }
            } else {
                for (int j = 0; j < kmax; ++j) {
                    __syncthreads();  // B1
                    __syncthreads();  // B2
                    __syncthreads();  // B3
                    __syncthreads();  // B4
                    __syncthreads();  // B5
                    const double alj = block_sum(0.0, red);           // B6, B7
                    const double bn = sqrt(block_sum(0.0, red));      // B8, B9
                    if (lane == 0) {
                        al[j] = alj;
                        be[j + 1] = bn;
                    }
                    __syncthreads();  // B10
                    const int k = j + 1;
                    const bool exhausted = bn <= 1e-14 * fmax(fabs(al[0]), 1e-300);
                    const bool check = exhausted || k == kmax || (k >= 3 && (k < 12 || (k & 1) == 0));
                    double stop = 0.0;
                    if (check) {
                        // lanes 0-31: lambda_min; lanes 32-63: lambda_max
                        const bool want_min = lane < 32;
                        const int sub = lane & 31;
                        double lo = INFINITY, hi = -INFINITY;
#pragma nounroll
                        for (int i = 0; i < k; ++i) {
                            const double rad = (i ? fabs(be[i]) : 0.0) + (i + 1 < k ? fabs(be[i + 1]) : 0.0);
                            lo = fmin(lo, al[i] - rad);
                            hi = fmax(hi, al[i] + rad);
                        }
                        const double pad = 1e-14 * fmax(fabs(lo), fabs(hi)) + 1e-300;
                        lo -= pad;
                        hi += pad;
#pragma nounroll
                        for (int it = 0; it < 14; ++it) {
                            const double w = hi - lo;
                            const double x = lo + w * (double)(sub + 1) / 33.0;
                            const int cnt = sturm(al, be, k, x);
                            const bool hitp = want_min ? (cnt >= 1) : (cnt >= k);
                            const unsigned long long mask = __ballot(hitp);
                            const unsigned int half_mask = want_min ? (unsigned int)mask : (unsigned int)(mask >> 32);
                            const int first = half_mask ? __ffs((int)half_mask) - 1 : 32;
                            const double nlo = lo + w * (double)first / 33.0;
                            const double nhi = first < 32 ? lo + w * (double)(first + 1) / 33.0 : hi;
                            if (w > 2e-16 * fmax(fabs(lo), fabs(hi))) {
                                lo = nlo;
                                hi = nhi;
                            }
                        }
                        const double th = 0.5 * (lo + hi);
                        const double res = exhausted ? 0.0 : fabs(bn) * backward_norm(al, be, k, th);
                        if (sub == 0) {
                            sres[want_min ? 0 : 2] = th;
                            sres[want_min ? 1 : 3] = res;
                        }
                        const double thmin = __shfl(th, 0, 64), thmax = __shfl(th, 32, 64);
                        const double rmin = __shfl(res, 0, 64), rmax = __shfl(res, 32, 64);
                        // residual bound below tol |theta|, or at the rounding level of C
                        const double rho = fmax(fabs(thmin), fabs(thmax));
                        const double floor_r = 2.2e-14 * rho;
                        const bool cmin = rmin <= fmax(a.tol * fabs(thmin), floor_r);
                        const bool cmax = rmax <= fmax(a.tol * fabs(thmax), floor_r);
                        const bool conv_now = exhausted || (cmin && (a.min_only || cmax));
                        if (conv_now) stop = 1.0;
                        else if (k == kmax) stop = 2.0;
                    } else if (k == kmax) {
                        stop = 2.0;
                    }
                    if (lane == 0) {
                        sres[4] = stop;
                        sres[5] = (double)k;
                    }
                    __syncthreads();  // B11
                    if (stop != 0.0) break;
                }
            }
            __syncthreads();
            lmin = sres[0];
            lmax = sres[2];
            conv = sres[4] == 1.0;
            const int k = (int)sres[5];
            iters = k;
            // dense block: roots measured from the shifted origin t0
            double dtpd = INFINITY, dtmd = -INFINITY;
            if (lmax > 0.0) dtmd = t0 - 1.0 / lmax;
            if (lmin < 0.0) dtpd = t0 - 1.0 / lmin;
            if (a.min_only) dtmd = NAN;  // lambda_max is not converged by design
            tm = isnan(dtmd) ? dtmd : fmax(tm, dtmd);
            if (dtpd <= tp) {
                tp = dtpd;
                hit = HIT_DENSE;
            }
            if (a.shift && !(lmin < 0.0 && dtpd > t0)) cert = 3;
            const bool need_vec = a.want_vec && hit == HIT_DENSE && isfinite(tp) && (a.ell == nullptr || tp < a.ell[chain]);
            if (need_vec && cert == 0) {
                // Ritz vector z = sum_j y_j q_j, y from the backward recurrence
                double zr = 0.0, y1 = 1.0, y0 = 0.0, ss = 0.0;
                for (int i = k - 1; i >= 0; --i) {
                    if (own) zr += y1 * Qg[(size_t)i * m + r];
                    ss += y1 * y1;
                    if (i >= 1) {
                        const double ym = ((lmin - al[i]) * y1 - (i + 1 < k ? be[i + 1] * y0 : 0.0)) / be[i];
                        y0 = y1;
                        y1 = ym;
                    }
                    if (ss > 1e280) {
                        const double sc = 1e-140;
                        y0 *= sc; y1 *= sc; ss *= sc * sc; zr *= sc;
                    }
                }
                zr *= 1.0 / sqrt(ss);
                __syncthreads();
                if (own && h == 0) slot[r] = zr;
                __syncthreads();
                // u = W^T z
                double uv = 0.0;
                if (own) {
                    const int c = r, mid = (R0w + m) >> 1;
                    const int rb = h == 0 ? R0w : mid, re = h == 0 ? mid : m;
                    for (int rr = rb; rr < re; ++rr)
                        if (rr >= c) uv += L[pk(rr, c)] * slot[rr];
                }
                uv += __shfl_xor(uv, 1, 64);
                __syncthreads();
                if (own && h == 0) {
                    a.u[(size_t)chain * a.ldu + r] = uv;
                    slot[r] = uv;
                }
                __syncthreads();
                if (own) {
                    double* U2 = a.U2 + (size_t)chain * a.ldu2;
                    const double ur = slot[r];
                    const int half = (r + 2) >> 1;
                    const int kb = h == 0 ? 0 : half, ke = h == 0 ? half : r + 1;
                    for (int cc = kb; cc < ke; ++cc) U2[pk(r, cc)] = (cc == r ? 1.0 : 2.0) * ur * slot[cc];
                }
            }
        }
    }
    if (t == 0) {
        if (st == SPEC_OK && cert) st = SPEC_CERT_FALLBACK;
        if (st == SPEC_NOT_INTERIOR) {
            tm = NAN;
            tp = NAN;
            hit = HIT_NONE;
        } else if (st == SPEC_OK && !a.membership_only) {
            if (!conv) st = SPEC_NOCONV;
            else if (isinf(tp) || isinf(tm)) st = SPEC_UNBOUNDED;
        }
        a.tm[chain] = tm;
        a.tp[chain] = tp;
        a.hit[chain] = hit;
        if (a.lam) {
            a.lam[4 * chain + 0] = lmin;
            a.lam[4 * chain + 1] = lmax;
            a.lam[4 * chain + 2] = (double)cert;
            a.lam[4 * chain + 3] = (double)iters;
        }
        a.status[chain] = st;
    }
}

size_t fused_lds_bytes(int m, int kmax) {
    const size_t P = (size_t)m * (m + 1) / 2;
    size_t scr = (size_t)2 * MAXH + 2 * (size_t)kmax + 1 + 16;
    if (scr < 304) scr = 304;
    return sizeof(double) * (P + scr);
}

int fused_threads(int m) {
    // one steering wave + 2m worker lanes in whole waves
    int t = 64 + ((2 * m + 63) / 64) * 64;
    if (t < 128) t = 128;
    return t;
}

hipError_t launch_line_fused(const FusedArgs& a, int nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    if (a.m > 2 * MAXH) return hipErrorInvalidValue;
    const size_t lds = fused_lds_bytes(a.m, a.kmax);
    if (lds > 163840) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_line_fused, dim3(nblocks), dim3(fused_threads(a.m)), lds, s, a);
    return hipGetLastError();
}

}  // namespace spec
