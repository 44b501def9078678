// Per-chain kernels of the line oracle (paper: Alg. INTERSECTION for
// Phi(t) = x + t v, Lemma "PEP and S cap C"; Alg. REFLECTION, Lemma
// "Gradient of det F").
//
// With F(x) = L L^T and W = L^{-1}, F(x) + t B(v) = L (I + t C) L^T with
// C = W B W^T, so the line leaves S at t+ = -1/lambda_min(C) and
// t- = -1/lambda_max(C) (the degree-one polynomial eigenvalue problem).
//
//   k_factor   one workgroup per chain: F (packed) in LDS, Cholesky, then the
//              triangular inverse W = L^{-1} in place; W to HBM.
//   k_lanczos  one workgroup per chain: Lanczos on C = W B W^T (three
//              matrix-vector products per step, W and B streamed from L2/HBM)
//              with full reorthogonalisation against the basis kept in LDS;
//              the extreme Ritz values of the tridiagonal T_k by multisection
//              of Sturm counts; stop when the residual bound beta_{k+1}|s_k|
//              of both extremes falls below tol |theta|.  Diagonal (polytope)
//              rows are handled by the ratio test.  For reflections the Ritz
//              vector z of lambda_min gives u = W^T z, a kernel vector of
//              F(x + t+ v), and vec(u u^T) is written for the normal GEMM.
#include "common.h"
#include "spec_kernels.h"

namespace spec {

// ----------------------------------------------------------------- factor

__global__ __launch_bounds__(256) void k_factor(int batch, int m, int md, int P, const double* __restrict__ FB,
                                                int ldfb, double* __restrict__ Wout, int ldw,
                                                int32_t* __restrict__ status) {
    extern __shared__ double lds[];
    double* L = lds;           // P
    double* tmp = lds + P;     // m
    const int c = blockIdx.x;
    if (c >= batch) return;
    const int t = threadIdx.x, nt = blockDim.x;
    const double* F = FB + (size_t)c * ldfb;
    for (int e = t; e < P; e += nt) L[e] = F[e];
    // diagonal (polytope) rows must be strictly positive
    int bad = 0;
    for (int j = t; j < md; j += nt) bad |= !(F[P + j] > 0.0);
    bad = __syncthreads_or(bad);

    // Cholesky, right-looking by columns, in place on the packed rows.
    for (int j = 0; j < m && !bad; ++j) {
        __syncthreads();
        const double d = L[pk(j, j)];
        if (!(d > 0.0)) { bad = 1; break; }  // uniform: every thread read the same value
        const double ljj = sqrt(d), inv = 1.0 / ljj;
        __syncthreads();
        for (int i = j + 1 + t; i < m; i += nt) L[pk(i, j)] *= inv;
        if (t == 0) L[pk(j, j)] = ljj;
        __syncthreads();
        for (int i = j + 1 + t; i < m; i += nt) {
            const double lij = L[pk(i, j)];
            double* row = L + pk(i, 0);
            for (int k = j + 1; k <= i; ++k) row[k] -= lij * L[pk(k, j)];
        }
    }
    if (bad) {
        if (t == 0) status[c] = SPEC_NOT_INTERIOR;
        return;
    }
    // W = L^{-1} in place: column j from the already inverted trailing block,
    // W[i][j] = -(1/L_jj) sum_{k=j+1..i} W[i][k] L[k][j].
    for (int j = m - 1; j >= 0; --j) {
        __syncthreads();
        for (int i = j + 1 + t; i < m; i += nt) tmp[i] = L[pk(i, j)];
        __syncthreads();
        const double wjj = 1.0 / L[pk(j, j)];
        for (int i = j + 1 + t; i < m; i += nt) {
            const double* row = L + pk(i, 0);
            double s = 0.0;
            for (int k = j + 1; k <= i; ++k) s += row[k] * tmp[k];
            L[pk(i, j)] = -wjj * s;
        }
        __syncthreads();
        if (t == 0) L[pk(j, j)] = wjj;
    }
    __syncthreads();
    double* Wc = Wout + (size_t)c * ldw;
    for (int e = t; e < P; e += nt) Wc[e] = L[e];
    if (t == 0) status[c] = SPEC_OK;
}

// ----------------------------------------------------------------- Lanczos

// Sturm count: number of eigenvalues of the k x k tridiagonal (al, be) below
// x, from the signs of the scaled characteristic-polynomial sequence.
__device__ inline int sturm_count(const double* al, const double* be, int k, double x) {
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
        const double b2 = i ? be[i] * be[i] : 0.0;
        d = (al[i] - x) - (i ? b2 / d : 0.0);
        if (d == 0.0) d = -1e-300;
        cnt += d < 0.0;
    }
    return cnt;
}

// Multisection by the 64 lanes of one wave for the smallest (want_min) or the
// largest eigenvalue of T_k inside [lo, hi]; returns the bracket.
__device__ inline void extreme_bracket(const double* al, const double* be, int k, bool want_min, double& lo,
                                       double& hi) {
    const int lane = threadIdx.x & 63;
    for (int it = 0; it < 12; ++it) {
        const double w = hi - lo;
        if (!(w > 2e-16 * fmax(fabs(lo), fabs(hi)))) break;
        const double x = lo + w * (double)(lane + 1) / 65.0;
        const int cnt = sturm_count(al, be, k, x);
        // want_min: first point with count >= 1; want_max: first with count >= k
        const bool hit = want_min ? (cnt >= 1) : (cnt >= k);
        const unsigned long long mask = __ballot(hit);
        const int first = mask ? __ffsll((long long)mask) - 1 : 64;
        const double nlo = lo + w * (double)first / 65.0;
        const double nhi = first < 64 ? lo + w * (double)(first + 1) / 65.0 : hi;
        lo = nlo;
        hi = nhi;
    }
}

// Eigenvector of T_k for an eigenvalue just outside the spectrum edge by two
// steps of inverse iteration with the shift sh (T - sh I is definite there,
// so the LDL^T of the Thomas algorithm needs no pivoting).  Single lane.
__device__ inline void tri_eigvec(const double* al, const double* be, int k, double sh, double* y,
                                  double* dwork) {
    for (int i = 0; i < k; ++i) y[i] = 1.0;
    for (int rep = 0; rep < 2; ++rep) {
        // forward elimination
        double d = al[0] - sh;
        if (d == 0.0) d = 1e-300;
        dwork[0] = d;
        for (int i = 1; i < k; ++i) {
            const double l = be[i] / dwork[i - 1];
            d = (al[i] - sh) - l * be[i];
            if (d == 0.0) d = 1e-300;
            dwork[i] = d;
            y[i] -= l * y[i - 1];
        }
        y[k - 1] /= dwork[k - 1];
        for (int i = k - 2; i >= 0; --i) y[i] = (y[i] - be[i + 1] * y[i + 1]) / dwork[i];
        double nrm = 0.0;
        for (int i = 0; i < k; ++i) nrm += y[i] * y[i];
        nrm = 1.0 / sqrt(nrm);
        for (int i = 0; i < k; ++i) y[i] *= nrm;
    }
}

struct LanczosShared {
    double* Q;     // kmax x mq basis
    double* vq;    // current q (alias of Q row j)
    double* va;    // m
    double* vb;    // m
    double* vc;    // m
    double* al;    // kmax
    double* be;    // kmax + 1 (be[0] unused)
    double* ymin;  // kmax
    double* ymax;  // kmax
    double* dw;    // 2 * kmax
    double* red;   // 16
};

// y = W^T x (W lower packed, global): y[k] = sum_{i >= k} W[i][k] x[i].
// Thread per column; rows walked from the first row of the thread's wave so
// that lanes of a wave read consecutive addresses.
__device__ inline void wt_x(const double* __restrict__ W, int m, const double* x, double* y) {
    const int t = threadIdx.x, nt = blockDim.x;
    for (int k = t; k < m; k += nt) {
        double s = 0.0;
        for (int i = k & ~63; i < m; ++i)
            if (i >= k) s += W[pk(i, k)] * x[i];
        y[k] = s;
    }
}

// y = M x for the lower rows of a packed matrix (strict when `strict`):
// y[r] = sum_{c <= r (c < r)} M[r][c] x[c].  One wave per row.
__device__ inline void lower_rows_x(const double* __restrict__ M, int m, const double* x, double* y, bool strict,
                                    bool accumulate) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int r = wid; r < m; r += nw) {
        const int len = strict ? r : r + 1;
        const double* row = M + pk(r, 0);
        double s = 0.0;
        for (int cc = lane; cc < len; cc += 64) s += row[cc] * x[cc];
        s = wave_sum(s);
        if (lane == 0) y[r] = accumulate ? y[r] + s : s;
    }
}

// y += sum_{i >= k} M[i][k] x[i] for a packed symmetric matrix (the upper
// triangle seen through the stored lower one), thread per column.
__device__ inline void sym_cols_x(const double* __restrict__ M, int m, const double* x, double* y) {
    const int t = threadIdx.x, nt = blockDim.x;
    for (int k = t; k < m; k += nt) {
        double s = 0.0;
        for (int i = k & ~63; i < m; ++i)
            if (i >= k) s += M[pk(i, k)] * x[i];
        y[k] += s;
    }
}

__global__ __launch_bounds__(256) void k_lanczos(LanczosArgs a) {
    extern __shared__ double lds[];
    const int c = blockIdx.x;
    if (c >= a.batch) return;
    const int t = threadIdx.x, nt = blockDim.x, wid = t >> 6, lane = t & 63;
    const int m = a.m, md = a.md, P = a.P;
    const int kmax = a.kmax < m ? a.kmax : m;
    const int mq = m | 1;
    LanczosShared S;
    S.Q = lds;
    S.va = S.Q + (size_t)kmax * mq;
    S.vb = S.va + m;
    S.vc = S.vb + m;
    S.al = S.vc + m;
    S.be = S.al + kmax;
    S.ymin = S.be + kmax + 1;
    S.ymax = S.ymin + kmax;
    S.dw = S.ymax + kmax;
    S.red = S.dw + 2 * kmax;
    __shared__ double sh_res[8];
    __shared__ int sh_flag[4];

    int32_t st = a.status[c];
    const double* Fd = a.FB + (size_t)c * a.ldfb + P;            // diagonal rows of F(x)
    const double* Bd = a.FB + (size_t)(a.brow0 + c) * a.ldfb + P; // diagonal rows of B(v)
    if (st == SPEC_NOT_INTERIOR) {
        if (t == 0) {
            a.tm[c] = NAN;
            a.tp[c] = NAN;
            a.hit[c] = HIT_NONE;
        }
        return;
    }
    // ---- diagonal rows: ratio test (polytope part of the LMI)
    double dtp = INFINITY, dtm = -INFINITY;
    int dj = -1;
    for (int j = t; j < md; j += nt) {
        const double r = Bd[j] / Fd[j];
        if (r < 0.0) {
            const double tt = -1.0 / r;
            if (tt < dtp) { dtp = tt; dj = j; }
        } else if (r > 0.0) {
            dtm = fmax(dtm, -1.0 / r);
        }
    }
    // reduce (min with index, max)
    {
        for (int o = 32; o > 0; o >>= 1) {
            const double otp = __shfl_xor(dtp, o, 64);
            const int oj = __shfl_xor(dj, o, 64);
            if (otp < dtp || (otp == dtp && oj >= 0 && (dj < 0 || oj < dj))) { dtp = otp; dj = oj; }
            dtm = fmax(dtm, __shfl_xor(dtm, o, 64));
        }
        __shared__ double rtp[4], rtm[4];
        __shared__ int rj[4];
        if (lane == 0) { rtp[wid] = dtp; rtm[wid] = dtm; rj[wid] = dj; }
        __syncthreads();
        dtp = INFINITY; dtm = -INFINITY; dj = -1;
        for (int w = 0; w < (nt >> 6); ++w) {
            if (rtp[w] < dtp || (rtp[w] == dtp && rj[w] >= 0 && (dj < 0 || rj[w] < dj))) { dtp = rtp[w]; dj = rj[w]; }
            dtm = fmax(dtm, rtm[w]);
        }
    }
    double tp = dtp, tm = dtm;
    int hit = dj >= 0 ? dj : HIT_NONE;  // >= 0: diagonal row; HIT_DENSE: dense block (set below)
    double lmin = 0.0, lmax = 0.0, l2 = 0.0;
    int iters = 0;
    bool conv = true;
    if (m > 0) {
        const double* W = a.W + (size_t)c * a.ldw;
        const double* B = a.FB + (size_t)(a.brow0 + c) * a.ldfb;
        // deterministic start vector with positive entries
        double* q0 = S.Q;
        double nrm = 0.0;
        for (int k = t; k < m; k += nt) {
            u4 h = philox10(u4{(uint32_t)k, 0x5eedu, 0u, 0x51a7u}, 0x2010u, 0x3817u);
            const double v = 0.5 + (double)(h.x >> 11) * (1.0 / 2097152.0);
            q0[k] = v;
            nrm += v * v;
        }
        nrm = block_sum(nrm, S.red);
        nrm = 1.0 / sqrt(nrm);
        for (int k = t; k < m; k += nt) q0[k] *= nrm;
        __syncthreads();
        int k = 0;  // number of basis vectors with completed (alpha, beta)
        double rmin = INFINITY, rmax = INFINITY;
        conv = false;
        for (int j = 0; j < kmax; ++j) {
            double* q = S.Q + (size_t)j * mq;
            // c = W B W^T q
            wt_x(W, m, q, S.va);
            __syncthreads();
            for (int r = t; r < m; r += nt) S.vb[r] = 0.0;
            __syncthreads();
            lower_rows_x(B, m, S.va, S.vb, false, true);
            __syncthreads();
            sym_cols_x(B, m, S.va, S.vb);  // adds the diagonal a second time:
            __syncthreads();
            for (int r = t; r < m; r += nt) S.vb[r] -= B[pk(r, r)] * S.va[r];
            __syncthreads();
            lower_rows_x(W, m, S.vb, S.vc, false, false);
            __syncthreads();
            double al = 0.0;
            for (int r = t; r < m; r += nt) al += q[r] * S.vc[r];
            al = block_sum(al, S.red);
            const double bej = j ? S.be[j] : 0.0;
            const double* qp = j ? S.Q + (size_t)(j - 1) * mq : q;
            for (int r = t; r < m; r += nt) S.vc[r] -= al * q[r] + bej * qp[r];
            __syncthreads();
            // full reorthogonalisation (classical Gram-Schmidt against q_0..q_j)
            for (int i = t; i <= j; i += nt) {
                const double* qi = S.Q + (size_t)i * mq;
                double h = 0.0;
                for (int r = 0; r < m; ++r) h += qi[r] * S.vc[r];
                S.dw[i] = h;
            }
            __syncthreads();
            for (int r = t; r < m; r += nt) {
                double s = S.vc[r];
                for (int i = 0; i <= j; ++i) s -= S.dw[i] * S.Q[(size_t)i * mq + r];
                S.vc[r] = s;
            }
            double bn = 0.0;
            for (int r = t; r < m; r += nt) bn += S.vc[r] * S.vc[r];
            bn = sqrt(block_sum(bn, S.red));
            if (t == 0) {
                S.al[j] = al;
                S.be[j + 1] = bn;
            }
            k = j + 1;
            __syncthreads();
            const double scale_c = fmax(fabs(S.al[0]), 1e-300);
            const bool exhausted = (bn <= 1e-14 * scale_c) || (k == m);
            const bool check = exhausted || k == kmax || (k >= 8 && (k % 4) == 0);
            if (check) {
                // extreme Ritz values and residual bounds on T_k
                if (wid < 2) {
                    double glo = INFINITY, ghi = -INFINITY;
                    for (int i = 0; i < k; ++i) {
                        const double rad = (i ? fabs(S.be[i]) : 0.0) + (i + 1 < k ? fabs(S.be[i + 1]) : 0.0);
                        glo = fmin(glo, S.al[i] - rad);
                        ghi = fmax(ghi, S.al[i] + rad);
                    }
                    const double pad = 1e-14 * fmax(fabs(glo), fabs(ghi)) + 1e-300;
                    double lo = glo - pad, hi = ghi + pad;
                    extreme_bracket(S.al, S.be, k, wid == 0, lo, hi);
                    if (lane == 0) {
                        double* y = wid == 0 ? S.ymin : S.ymax;
                        const double shift = wid == 0 ? lo - 1e-15 * fabs(lo) : hi + 1e-15 * fabs(hi);
                        tri_eigvec(S.al, S.be, k, shift, y, S.dw + (wid == 0 ? 0 : kmax));
                        const double theta = 0.5 * (lo + hi);
                        sh_res[wid * 2] = theta;
                        sh_res[wid * 2 + 1] = exhausted ? 0.0 : fabs(bn * y[k - 1]);
                    }
                }
                __syncthreads();
                lmin = sh_res[0];
                lmax = sh_res[2];
                rmin = sh_res[1];
                rmax = sh_res[3];
                const double rho = fmax(fabs(lmin), fabs(lmax));
                conv = exhausted || (rmin <= a.tol * fmax(fabs(lmin), 1e-4 * rho) &&
                                     rmax <= a.tol * fmax(fabs(lmax), 1e-4 * rho));
                if (conv || k == kmax) break;
            }
            // next basis vector
            double* qn = S.Q + (size_t)(j + 1) * mq;
            const double ib = 1.0 / bn;
            for (int r = t; r < m; r += nt) qn[r] = S.vc[r] * ib;
            __syncthreads();
        }
        iters = k;
        // dense block contributions
        if (lmax > 0.0) tm = fmax(tm, -1.0 / lmax);
        if (lmin < 0.0) {
            const double tt = -1.0 / lmin;
            if (tt <= tp) { tp = tt; hit = HIT_DENSE; }
        }
        // second smallest Ritz value (multiplicity test), only for reflections
        const bool need_vec = a.want_vec && hit == HIT_DENSE && isfinite(tp) && (a.ell == nullptr || tp < a.ell[c]);
        if (need_vec) {
            if (wid == 0 && k > 1) {
                double glo = lmin, ghi = lmax + fabs(lmax) * 1e-14 + 1e-300;
                // bracket the second eigenvalue: first point with count >= 2
                double lo = glo, hi = ghi;
                for (int it = 0; it < 12; ++it) {
                    const double w = hi - lo;
                    if (!(w > 2e-16 * fmax(fabs(lo), fabs(hi)))) break;
                    const double x = lo + w * (double)(lane + 1) / 65.0;
                    const int cnt = sturm_count(S.al, S.be, k, x);
                    const unsigned long long mask = __ballot(cnt >= 2);
                    const int first = mask ? __ffsll((long long)mask) - 1 : 64;
                    const double nlo = lo + w * (double)first / 65.0;
                    const double nhi = first < 64 ? lo + w * (double)(first + 1) / 65.0 : hi;
                    lo = nlo;
                    hi = nhi;
                }
                if (lane == 0) sh_res[4] = 0.5 * (lo + hi);
            }
            __syncthreads();
            l2 = k > 1 ? sh_res[4] : INFINITY;
            // z = Q s_min, u = W^T z
            for (int r = t; r < m; r += nt) {
                double s = 0.0;
                for (int i = 0; i < k; ++i) s += S.ymin[i] * S.Q[(size_t)i * mq + r];
                S.va[r] = s;
            }
            __syncthreads();
            wt_x(W, m, S.va, S.vb);
            __syncthreads();
            double* u = a.u + (size_t)c * a.ldu;
            for (int r = t; r < m; r += nt) u[r] = S.vb[r];
            double* U2 = a.U2 + (size_t)c * a.ldu2;
            for (int r = wid; r < m; r += (nt >> 6)) {
                const double ur = S.vb[r];
                for (int cc = lane; cc <= r; cc += 64) U2[pk(r, cc)] = (cc == r ? 1.0 : 2.0) * ur * S.vb[cc];
            }
        }
    }
    if (t == 0) {
        if (st == SPEC_OK && !conv) st = SPEC_NOCONV;
        if (st == SPEC_OK && (isinf(tp) || isinf(tm))) st = SPEC_UNBOUNDED;
        a.tm[c] = tm;
        a.tp[c] = tp;
        a.hit[c] = hit;
        if (a.lam) {
            a.lam[4 * c + 0] = lmin;
            a.lam[4 * c + 1] = lmax;
            a.lam[4 * c + 2] = l2;
            a.lam[4 * c + 3] = (double)iters;
        }
        a.status[c] = st;
    }
}

size_t lanczos_lds_bytes(int m, int kmax) {
    const int km = kmax < m ? kmax : m;
    const int mq = m | 1;
    return sizeof(double) * ((size_t)km * mq + 3 * (size_t)m + 2 * (size_t)km + 1 + 2 * (size_t)km +
                             2 * (size_t)km + 16);
}

size_t factor_lds_bytes(int m) { return sizeof(double) * ((size_t)m * (m + 1) / 2 + (size_t)m); }

hipError_t launch_factor(int batch, int m, int md, int P, const double* FB, int ldfb, double* W, int ldw,
                         int32_t* status, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    const size_t lds = factor_lds_bytes(m);
    hipLaunchKernelGGL(k_factor, dim3(batch), dim3(256), lds, s, batch, m, md, P, FB, ldfb, W, ldw, status);
    return hipGetLastError();
}

hipError_t launch_lanczos(const LanczosArgs& a, hipStream_t s) {
    if (a.batch <= 0) return hipSuccess;
    const size_t lds = lanczos_lds_bytes(a.m, a.kmax);
    hipLaunchKernelGGL(k_lanczos, dim3(a.batch), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace spec
