/*
 * oracle.c -- plain, slow, FP64 CPU reference ("the oracle") of the boundary
 * oracle of Chalkis et al., "Efficient Sampling from Feasible Sets of SDPs and
 * Volume Approximation" (arXiv:2010.03817), and of the walks built on it.
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
 * baseline of the benchmark use this file.  It shares no code, header, table
 * or helper with the HIP path, and the HIP path never loads it.
 *
 * Style: straight loops, IEEE double, no BLAS, no blocking or fusion; every
 * routine cites the passage of the paper it follows.  Compile with
 * -O2 -fno-fast-math -ffp-contract=off.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct orc_lmi {
    int n, nb;
    int* m;      /* block sizes */
    int* kind;   /* ORC_DENSE / ORC_DIAG */
    double** A;  /* per block: (n+1)*m*m or (n+1)*m */
};

/* ------------------------------------------------------------------------ */
/* Instance                                                                  */
/* ------------------------------------------------------------------------ */

/* The LMI F(x) = A0 + sum_i x_i A_i of eq. (1), stored block by block; a
 * block-diagonal LMI is the same spectrahedron as its dense form. */
int orc_create(int n, int nb, const int* bs, const int* kind, const double* A, orc_lmi** out) {
    if (n < 1 || nb < 1 || !bs || !kind || !A || !out) return ORC_EINVAL;
    orc_lmi* h = (orc_lmi*)calloc(1, sizeof(orc_lmi));
    if (!h) return ORC_ENOMEM;
    h->n = n;
    h->nb = nb;
    h->m = (int*)malloc(sizeof(int) * nb);
    h->kind = (int*)malloc(sizeof(int) * nb);
    h->A = (double**)calloc(nb, sizeof(double*));
    const double* src = A;
    for (int b = 0; b < nb; b++) {
        if (bs[b] < 1 || (kind[b] != ORC_DENSE && kind[b] != ORC_DIAG)) { orc_destroy(h); return ORC_EINVAL; }
        h->m[b] = bs[b];
        h->kind[b] = kind[b];
        size_t cnt = (size_t)(n + 1) * bs[b] * (kind[b] == ORC_DENSE ? bs[b] : 1);
        h->A[b] = (double*)malloc(sizeof(double) * cnt);
        memcpy(h->A[b], src, sizeof(double) * cnt);
        src += cnt;
    }
    *out = h;
    return ORC_OK;
}

void orc_destroy(orc_lmi* h) {
    if (!h) return;
    if (h->A)
        for (int b = 0; b < h->nb; b++) free(h->A[b]);
    free(h->A);
    free(h->m);
    free(h->kind);
    free(h);
}

/* out = c0*A0 + sum_i y_i A_i for one block (dense: m*m, diag: m). */
static void combine(const orc_lmi* h, int b, double c0, const double* y, double* out) {
    int m = h->m[b];
    size_t sz = (size_t)m * (h->kind[b] == ORC_DENSE ? m : 1);
    const double* A = h->A[b];
    for (size_t e = 0; e < sz; e++) out[e] = c0 * A[e];
    for (int i = 0; i < h->n; i++) {
        const double* Ai = A + (size_t)(i + 1) * sz;
        double yi = y[i];
        if (yi == 0.0) continue;
        for (size_t e = 0; e < sz; e++) out[e] += yi * Ai[e];
    }
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra                                                      */
/* ------------------------------------------------------------------------ */

/* Cholesky-Banachiewicz, row by row.  Returns 0 if every pivot is strictly
 * positive (F is positive definite), else (index of the failing pivot + 1).
 * This is the membership test of Alg. MEMBERSHIP read as strict definiteness. */
static int cholesky(int m, const double* F, double* L) {
    memset(L, 0, sizeof(double) * (size_t)m * m);
    for (int i = 0; i < m; i++) {
        for (int j = 0; j <= i; j++) {
            double s = F[(size_t)i * m + j];
            for (int k = 0; k < j; k++) s -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
            if (i == j) {
                if (!(s > 0.0)) return i + 1;
                L[(size_t)i * m + i] = sqrt(s);
            } else {
                L[(size_t)i * m + j] = s / L[(size_t)j * m + j];
            }
        }
    }
    return 0;
}

/* C = L^{-1} B L^{-T}: forward substitution on the columns of B, then on the
 * rows of the result; symmetrised.  With F = L L^T, F + tB = L (I + tC) L^T,
 * so det(F + tB) = det(F) prod_k (1 + t lambda_k(C)) (Lemma "PEP and S cap C"
 * for a degree-one curve). */
static void congruence(int m, const double* L, const double* B, double* C, double* tmp) {
    /* tmp = L^{-1} B */
    for (int c = 0; c < m; c++)
        for (int i = 0; i < m; i++) {
            double s = B[(size_t)i * m + c];
            for (int k = 0; k < i; k++) s -= L[(size_t)i * m + k] * tmp[(size_t)k * m + c];
            tmp[(size_t)i * m + c] = s / L[(size_t)i * m + i];
        }
    /* C^T = L^{-1} tmp^T, i.e. C[r][i] solves row r of tmp */
    for (int r = 0; r < m; r++)
        for (int i = 0; i < m; i++) {
            double s = tmp[(size_t)r * m + i];
            for (int k = 0; k < i; k++) s -= L[(size_t)i * m + k] * C[(size_t)r * m + k];
            C[(size_t)r * m + i] = s / L[(size_t)i * m + i];
        }
    for (int i = 0; i < m; i++)
        for (int j = 0; j < i; j++) {
            double a = 0.5 * (C[(size_t)i * m + j] + C[(size_t)j * m + i]);
            C[(size_t)i * m + j] = a;
            C[(size_t)j * m + i] = a;
        }
}

/* Cyclic Jacobi eigenvalue method (row-cyclic sweeps over p<q, Rutishauser's
 * stable rotation).  A is overwritten (its diagonal holds the eigenvalues);
 * V (nullable) accumulates eigenvectors as columns.  Returns the number of
 * sweeps, or -1 if 50 sweeps did not reduce the off-diagonal Frobenius norm
 * below 1e-15 of the full norm. */
static int jacobi(int m, double* A, double* V) {
    if (V) {
        memset(V, 0, sizeof(double) * (size_t)m * m);
        for (int i = 0; i < m; i++) V[(size_t)i * m + i] = 1.0;
    }
    double fro = 0.0;
    for (size_t e = 0; e < (size_t)m * m; e++) fro += A[e] * A[e];
    fro = sqrt(fro);
    for (int sweep = 0; sweep <= 50; sweep++) {
        double off = 0.0;
        for (int p = 0; p < m; p++)
            for (int q = 0; q < m; q++)
                if (p != q) off += A[(size_t)p * m + q] * A[(size_t)p * m + q];
        off = sqrt(off);
        if (off <= 1e-15 * fro || off == 0.0) return sweep;
        if (sweep == 50) break;
        for (int p = 0; p < m - 1; p++)
            for (int q = p + 1; q < m; q++) {
                double apq = A[(size_t)p * m + q];
                if (fabs(apq) < 1e-300) continue;
                double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t;
                if (fabs(theta) > 1e150)
                    t = 0.5 / theta;
                else
                    t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int r = 0; r < m; r++) {
                    double arp = A[(size_t)r * m + p], arq = A[(size_t)r * m + q];
                    A[(size_t)r * m + p] = c * arp - s * arq;
                    A[(size_t)r * m + q] = s * arp + c * arq;
                }
                for (int r = 0; r < m; r++) {
                    double apr = A[(size_t)p * m + r], aqr = A[(size_t)q * m + r];
                    A[(size_t)p * m + r] = c * apr - s * aqr;
                    A[(size_t)q * m + r] = s * apr + c * aqr;
                }
                A[(size_t)p * m + p] = app - t * apq;
                A[(size_t)q * m + q] = aqq + t * apq;
                A[(size_t)p * m + q] = 0.0;
                A[(size_t)q * m + p] = 0.0;
                if (V)
                    for (int r = 0; r < m; r++) {
                        double vrp = V[(size_t)r * m + p], vrq = V[(size_t)r * m + q];
                        V[(size_t)r * m + p] = c * vrp - s * vrq;
                        V[(size_t)r * m + q] = s * vrp + c * vrq;
                    }
            }
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10                                                             */
/* ------------------------------------------------------------------------ */

/* Counter-based generator of Salmon, Moraes, Dror and Shaw ("Parallel random
 * numbers: as easy as 1, 2, 3", SC'11): ten rounds of the Philox S-box on a
 * 4x32-bit counter with a 2x32-bit key bumped by the Weyl constants. */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draw tags (fourth counter word, low byte); the phase of a volume run goes
 * in the next byte. */
enum { TAG_DIR = 1, TAG_LEN = 2, TAG_POS = 3, TAG_COORD = 4, TAG_MOM = 5, TAG_GAUSS0 = 6 };

/* Two uniforms in (0,1) with 53 random bits each from one Philox block. */
static void uniforms2(uint32_t a, uint32_t b, uint32_t c, uint32_t d, double u[2]) {
    u[0] = ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * (1.0 / 9007199254740992.0);
    u[1] = ((double)(c >> 5) * 67108864.0 + (double)(d >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

static void draw_u2(uint64_t seed, uint32_t chain, uint32_t step, uint32_t draw, uint32_t tag, double u[2]) {
    uint32_t ctr[4] = {chain, step, draw, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox(ctr, key, w);
    uniforms2(w[0], w[1], w[2], w[3], u);
}

/* k standard normals by Box-Muller (both outputs of each pair used). */
static void draw_normals(uint64_t seed, uint32_t chain, uint32_t step, uint32_t tag, int k, double* g) {
    const double two_pi = 6.283185307179586476925286766559;
    for (int d = 0; 2 * d < k; d++) {
        double u[2];
        draw_u2(seed, chain, step, (uint32_t)d, tag, u);
        double r = sqrt(-2.0 * log(u[0]));
        g[2 * d] = r * cos(two_pi * u[1]);
        if (2 * d + 1 < k) g[2 * d + 1] = r * sin(two_pi * u[1]);
    }
}

/* ------------------------------------------------------------------------ */
/* Boundary oracle                                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *F, *B, *L, *C, *T, *V;  /* m*m each, sized for the largest block */
    double *w;                      /* n */
} scratch;

static int max_block(const orc_lmi* h) {
    int mm = 1;
    for (int b = 0; b < h->nb; b++) if (h->m[b] > mm) mm = h->m[b];
    return mm;
}

static int scratch_alloc(const orc_lmi* h, scratch* s) {
    size_t mm = (size_t)max_block(h);
    s->F = (double*)malloc(sizeof(double) * mm * mm);
    s->B = (double*)malloc(sizeof(double) * mm * mm);
    s->L = (double*)malloc(sizeof(double) * mm * mm);
    s->C = (double*)malloc(sizeof(double) * mm * mm);
    s->T = (double*)malloc(sizeof(double) * mm * mm);
    s->V = (double*)malloc(sizeof(double) * mm * mm);
    s->w = (double*)malloc(sizeof(double) * (size_t)h->n);
    return (s->F && s->B && s->L && s->C && s->T && s->V && s->w) ? 0 : -1;
}

static void scratch_free(scratch* s) {
    free(s->F); free(s->B); free(s->L); free(s->C); free(s->T); free(s->V); free(s->w);
}

int orc_membership(const orc_lmi* h, int batch, const double* x, int8_t* interior) {
    if (!h || batch < 0 || (batch && (!x || !interior))) return ORC_EINVAL;
    scratch s;
    if (scratch_alloc(h, &s)) { scratch_free(&s); return ORC_ENOMEM; }
    for (int e = 0; e < batch; e++) {
        const double* xe = x + (size_t)e * h->n;
        int ok = 1;
        for (int b = 0; b < h->nb && ok; b++) {
            combine(h, b, 1.0, xe, s.F);
            if (h->kind[b] == ORC_DENSE) ok = cholesky(h->m[b], s.F, s.L) == 0;
            else for (int j = 0; j < h->m[b]; j++) if (!(s.F[j] > 0.0)) ok = 0;
        }
        interior[e] = (int8_t)ok;
    }
    scratch_free(&s);
    return ORC_OK;
}

/* Result of the line oracle for one element, with what reflection needs. */
typedef struct {
    double tp, tm;
    int bplus;        /* block attaining t+ (-1 if none) */
    int jplus;        /* for a DIAG block: entry attaining t+ */
    int status;
    int degenerate;   /* lambda_min of the hit block has numerical multiplicity */
    int tie;          /* two blocks attain t+ */
} line_res;

/* Alg. INTERSECTION for the line Phi(t) = x + t v (degree one):
 * per dense block, lambda(C) with C = L^{-1} B(v) L^{-T}; t+ = -1/lambda_min
 * (lambda_min < 0), t- = -1/lambda_max (lambda_max > 0); per diagonal entry
 * the ratio B_jj / F_jj.  The overall interval is the intersection over
 * blocks.  If want_vec, the eigenvector of the block attaining t+ is mapped
 * back to u = L^{-T} z (a kernel vector of F(x + t+ v)) and written to u. */
static line_res line_oracle(const orc_lmi* h, const double* x, const double* v, scratch* s,
                            double* u_out) {
    line_res r = {INFINITY, -INFINITY, -1, -1, ORC_OK, 0, 0};
    for (int b = 0; b < h->nb; b++) {
        int m = h->m[b];
        combine(h, b, 1.0, x, s->F);
        combine(h, b, 0.0, v, s->B);
        if (h->kind[b] == ORC_DIAG) {
            for (int j = 0; j < m; j++) {
                if (!(s->F[j] > 0.0)) { r.status = ORC_NOT_INTERIOR; return r; }
                double c = s->B[j] / s->F[j];
                if (c < 0.0) {
                    double t = -1.0 / c;
                    if (t < r.tp) { r.tp = t; r.bplus = b; r.jplus = j; r.tie = 0; }
                    else if (t == r.tp) r.tie = 1;
                } else if (c > 0.0) {
                    double t = -1.0 / c;
                    if (t > r.tm) r.tm = t;
                }
            }
            continue;
        }
        if (cholesky(m, s->F, s->L) != 0) { r.status = ORC_NOT_INTERIOR; return r; }
        congruence(m, s->L, s->B, s->C, s->T);
        int sw = jacobi(m, s->C, u_out ? s->V : NULL);
        if (sw < 0) r.status = ORC_NOCONV;
        int imin = 0, imax = 0;
        for (int k = 1; k < m; k++) {
            if (s->C[(size_t)k * m + k] < s->C[(size_t)imin * m + imin]) imin = k;
            if (s->C[(size_t)k * m + k] > s->C[(size_t)imax * m + imax]) imax = k;
        }
        double lmin = s->C[(size_t)imin * m + imin], lmax = s->C[(size_t)imax * m + imax];
        if (lmax > 0.0) {
            double t = -1.0 / lmax;
            if (t > r.tm) r.tm = t;
        }
        if (lmin < 0.0) {
            double t = -1.0 / lmin;
            if (t <= r.tp) {
                r.tie = (t == r.tp);
                r.tp = t;
                r.bplus = b;
                r.jplus = -1;
                double l2 = INFINITY;
                for (int k = 0; k < m; k++)
                    if (k != imin && s->C[(size_t)k * m + k] < l2) l2 = s->C[(size_t)k * m + k];
                r.degenerate = (m > 1 && fabs(l2 - lmin) <= 1e-10 * fabs(lmin));
                if (u_out) {
                    /* u = L^{-T} z: back substitution on L^T u = z */
                    for (int i = m - 1; i >= 0; i--) {
                        double acc = s->V[(size_t)i * m + imin];
                        for (int k = i + 1; k < m; k++) acc -= s->L[(size_t)k * m + i] * u_out[k];
                        u_out[i] = acc / s->L[(size_t)i * m + i];
                    }
                }
            }
        }
    }
    if (r.status == ORC_OK && (isinf(r.tp) || isinf(r.tm))) r.status = ORC_UNBOUNDED;
    return r;
}

int orc_intersect(const orc_lmi* h, int batch, const double* x, const double* v,
                  double* tm, double* tp, int32_t* st) {
    if (!h || batch < 0 || (batch && (!x || !v || !tm || !tp || !st))) return ORC_EINVAL;
    scratch s;
    if (scratch_alloc(h, &s)) { scratch_free(&s); return ORC_ENOMEM; }
    for (int e = 0; e < batch; e++) {
        line_res r = line_oracle(h, x + (size_t)e * h->n, v + (size_t)e * h->n, &s, NULL);
        if (r.status == ORC_NOT_INTERIOR) { tm[e] = NAN; tp[e] = NAN; }
        else { tm[e] = r.tm; tp[e] = r.tp; }
        st[e] = r.status;
    }
    scratch_free(&s);
    return ORC_OK;
}

/* Membership of the pencil point F(x) + t B(v) = F(x + t v) over every block
 * (strict definiteness, as orc_membership).  Fx, Bv hold the blocks of F(x)
 * and B(v) back to back (block b at offset off[b]); P is scratch. */
static int pencil_member(const orc_lmi* h, const double* Fx, const double* Bv, const size_t* off,
                         double t, double* P, double* L) {
    for (int b = 0; b < h->nb; b++) {
        int m = h->m[b];
        size_t sz = h->kind[b] == ORC_DENSE ? (size_t)m * m : (size_t)m;
        for (size_t k = 0; k < sz; k++) P[k] = Fx[off[b] + k] + t * Bv[off[b] + k];
        if (h->kind[b] == ORC_DENSE) {
            if (cholesky(m, P, L) != 0) return 0;
        } else {
            for (int j = 0; j < m; j++) if (!(P[j] > 0.0)) return 0;
        }
    }
    return 1;
}

/* End of the feasible interval along +v from membership alone: the definition
 * t+ = sup{t >= 0 : F(x + s v) > 0 for all s in [0, t]} of Lemma "PEP and S
 * cap C".  S is convex, so the feasible t form one interval and bisection on
 * membership finds its end: from the guess g (1 if g is not a positive
 * finite number) the bracket [lo, hi] is grown by doubling or shrunk by
 * halving until lo is a member and hi is not, then halved until its midpoint
 * equals an end (lo and hi adjacent doubles); returns lo, the last member.
 * INFINITY when every t up to 1e300 is a member. */
static double bisect_end(const orc_lmi* h, const double* Fx, const double* Bv, const size_t* off, double g,
                         double* P, double* L) {
    double lo = 0.0, hi = (g > 0.0 && isfinite(g)) ? g : 1.0;
    if (pencil_member(h, Fx, Bv, off, hi, P, L)) {
        do {
            lo = hi;
            hi = 2.0 * hi;
            if (hi > 1e300) return INFINITY;
        } while (pencil_member(h, Fx, Bv, off, hi, P, L));
    } else {
        for (;;) {
            double half = 0.5 * hi;
            if (!(half > 0.0)) return 0.0;
            if (pencil_member(h, Fx, Bv, off, half, P, L)) { lo = half; break; }
            hi = half;
        }
    }
    for (;;) {
        double mid = lo + 0.5 * (hi - lo);
        if (!(mid > lo && mid < hi)) break;
        if (pencil_member(h, Fx, Bv, off, mid, P, L)) lo = mid;
        else hi = mid;
    }
    return lo;
}

int orc_line_bisect(const orc_lmi* h, int batch, const double* x, const double* v, const double* guess,
                    double* tm, double* tp, int32_t* st) {
    if (!h || batch < 0 || (batch && (!x || !v || !tm || !tp || !st))) return ORC_EINVAL;
    size_t* off = (size_t*)malloc(sizeof(size_t) * (size_t)h->nb);
    size_t tot = 0;
    for (int b = 0; b < h->nb; b++) {
        off[b] = tot;
        tot += h->kind[b] == ORC_DENSE ? (size_t)h->m[b] * h->m[b] : (size_t)h->m[b];
    }
    size_t mm = (size_t)max_block(h);
    double* Fx = (double*)malloc(sizeof(double) * tot);
    double* Bv = (double*)malloc(sizeof(double) * tot);
    double* Bn = (double*)malloc(sizeof(double) * tot);
    double* P = (double*)malloc(sizeof(double) * mm * mm);
    double* L = (double*)malloc(sizeof(double) * mm * mm);
    if (!off || !Fx || !Bv || !Bn || !P || !L) {
        free(off); free(Fx); free(Bv); free(Bn); free(P); free(L);
        return ORC_ENOMEM;
    }
    for (int e = 0; e < batch; e++) {
        const double* xe = x + (size_t)e * h->n;
        const double* ve = v + (size_t)e * h->n;
        for (int b = 0; b < h->nb; b++) {
            combine(h, b, 1.0, xe, Fx + off[b]);
            combine(h, b, 0.0, ve, Bv + off[b]);
        }
        for (size_t k = 0; k < tot; k++) Bn[k] = -Bv[k];
        if (!pencil_member(h, Fx, Bv, off, 0.0, P, L)) {
            tm[e] = NAN; tp[e] = NAN; st[e] = ORC_NOT_INTERIOR;
            continue;
        }
        double gp = guess ? guess[2 * e + 1] : 1.0, gm = guess ? -guess[2 * e] : 1.0;
        tp[e] = bisect_end(h, Fx, Bv, off, gp, P, L);
        tm[e] = -bisect_end(h, Fx, Bn, off, gm, P, L);
        st[e] = (isinf(tp[e]) || isinf(tm[e])) ? ORC_UNBOUNDED : ORC_OK;
    }
    free(off); free(Fx); free(Bv); free(Bn); free(P); free(L);
    return ORC_OK;
}

/* Normal at the hit point from Lemma "Gradient of det F": grad det F(p) is a
 * multiple of (u^T A_1 u, ..., u^T A_n u), u in ker F(p); the scale and
 * orientation are dropped (the vector is normalised). For a diagonal entry j
 * the gradient of F_jj is (A_1[j], ..., A_n[j]). */
static void normal_at(const orc_lmi* h, int b, int j, const double* u, double* w) {
    int m = h->m[b], n = h->n;
    if (h->kind[b] == ORC_DIAG) {
        for (int i = 0; i < n; i++) w[i] = h->A[b][(size_t)(i + 1) * m + j];
        return;
    }
    for (int i = 0; i < n; i++) {
        const double* Ai = h->A[b] + (size_t)(i + 1) * m * m;
        double acc = 0.0;
        for (int r = 0; r < m; r++) {
            double row = 0.0;
            for (int c = 0; c < m; c++) row += Ai[(size_t)r * m + c] * u[c];
            acc += u[r] * row;
        }
        w[i] = acc;
    }
}

/* Specular reflection of eq. (reflection): s = d - 2 <d, w_hat> w_hat, with
 * w_hat oriented outward (<d, w_hat> >= 0).  Returns 1 if w = 0. */
static int reflect_dir(int n, const double* d, double* w, double* s) {
    double nw = 0.0;
    for (int i = 0; i < n; i++) nw += w[i] * w[i];
    nw = sqrt(nw);
    if (!(nw > 0.0)) {
        for (int i = 0; i < n; i++) s[i] = d[i];
        return 1;
    }
    double dw = 0.0;
    for (int i = 0; i < n; i++) { w[i] /= nw; dw += d[i] * w[i]; }
    if (dw < 0.0) {
        for (int i = 0; i < n; i++) w[i] = -w[i];
        dw = -dw;
    }
    for (int i = 0; i < n; i++) s[i] = d[i] - 2.0 * dw * w[i];
    return 0;
}

int orc_reflect(const orc_lmi* h, int batch, const double* x, const double* v,
                double* tp, double* s_out, double* w_out, int32_t* st) {
    if (!h || batch < 0 || (batch && (!x || !v || !tp || !s_out || !st))) return ORC_EINVAL;
    scratch s;
    if (scratch_alloc(h, &s)) { scratch_free(&s); return ORC_ENOMEM; }
    double* u = (double*)malloc(sizeof(double) * (size_t)max_block(h));
    int n = h->n;
    for (int e = 0; e < batch; e++) {
        const double* xe = x + (size_t)e * n;
        const double* ve = v + (size_t)e * n;
        double* se = s_out + (size_t)e * n;
        line_res r = line_oracle(h, xe, ve, &s, u);
        int status = r.status;
        if (status == ORC_NOT_INTERIOR) {
            tp[e] = NAN;
            for (int i = 0; i < n; i++) { se[i] = NAN; if (w_out) w_out[(size_t)e * n + i] = NAN; }
        } else if (isinf(r.tp)) {
            tp[e] = r.tp;
            for (int i = 0; i < n; i++) { se[i] = ve[i]; if (w_out) w_out[(size_t)e * n + i] = 0.0; }
        } else {
            tp[e] = r.tp;
            normal_at(h, r.bplus, r.jplus, u, s.w);
            int zero = reflect_dir(n, ve, s.w, se);
            if (w_out) memcpy(w_out + (size_t)e * n, s.w, sizeof(double) * n);
            if (status == ORC_OK && (zero || r.degenerate || r.tie)) status = ORC_NONSMOOTH;
        }
        st[e] = status;
    }
    free(u);
    scratch_free(&s);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Degree-two curves                                                         */
/* ------------------------------------------------------------------------ */

/* Smallest positive root of 1 + a s + b s^2 (INFINITY if none). */
static double first_root_q(double a, double b) {
    double disc = a * a - 4.0 * b;
    if (disc < 0.0) return INFINITY;
    double den = -a + sqrt(disc);
    if (!(den > 0.0)) return INFINITY;
    return 2.0 / den;
}

/* First positive root of det Q(t), Q(t) = Q0 + t Q1 + t^2 Q2, Q0 > 0, for one
 * dense block (the polynomial eigenvalue problem of eq. (PEP) with d = 2).
 * Certified stepping: at tau with Q(tau) = L L^T, Q(tau + s) =
 * L (I + s D1 + s^2 D2) L^T with D1 = L^{-1}(Q1 + 2 tau Q2)L^{-T},
 * D2 = L^{-1} Q2 L^{-T}, and by Weyl's inequality the matrix stays definite
 * while 1 + s lambda_min(D1) + s^2 lambda_min(D2) > 0.  Step to that bound
 * until the step is negligible; the limit is the smallest positive root
 * (Lemma "PEP and S cap C").  Returns INFINITY if none below the horizon. */
static double curve2_dense(int m, const double* Q0, const double* Q1, const double* Q2,
                           double horizon, scratch* s, int* status, int* iters) {
    double* Qt = s->F;
    double* Q1e = s->B;
    double tau = 0.0;
    for (int it = 0; it < 200; it++) {
        *iters = it + 1;
        for (size_t e = 0; e < (size_t)m * m; e++) Qt[e] = Q0[e] + tau * Q1[e] + tau * tau * Q2[e];
        if (cholesky(m, Qt, s->L) != 0) {
            if (it == 0) { *status = ORC_NOT_INTERIOR; return NAN; }
            return tau; /* definiteness lost at rounding level: converged */
        }
        for (size_t e = 0; e < (size_t)m * m; e++) Q1e[e] = Q1[e] + 2.0 * tau * Q2[e];
        congruence(m, s->L, Q1e, s->C, s->T);
        if (jacobi(m, s->C, NULL) < 0) *status = ORC_NOCONV;
        double a = INFINITY;
        for (int k = 0; k < m; k++) if (s->C[(size_t)k * m + k] < a) a = s->C[(size_t)k * m + k];
        congruence(m, s->L, Q2, s->C, s->T);
        if (jacobi(m, s->C, NULL) < 0) *status = ORC_NOCONV;
        double b = INFINITY;
        for (int k = 0; k < m; k++) if (s->C[(size_t)k * m + k] < b) b = s->C[(size_t)k * m + k];
        double step = first_root_q(a, b);
        if (isinf(step)) return INFINITY;
        double next = tau + step;
        if (next > horizon) return INFINITY;
        if (step <= 1e-15 * next) return next;
        tau = next;
    }
    *status = ORC_NOCONV;
    return tau;
}

/* Smallest positive root of c0 + c1 t + c2 t^2 with c0 > 0 (one diagonal entry). */
static double first_root_scalar(double c0, double c1, double c2) {
    /* divide by c0: 1 + (c1/c0) t + (c2/c0) t^2 */
    return first_root_q(c1 / c0, c2 / c0);
}

/* First positive root of det Q over all blocks; writes the block and entry. */
static double curve2_first(const orc_lmi* h, const double* coef, double sign1, double horizon,
                           scratch* s, double* Q0, double* Q1, double* Q2, int* status,
                           int* iters, int* bhit, int* jhit) {
    int n = h->n;
    double best = INFINITY;
    *bhit = -1;
    *jhit = -1;
    double* y = (double*)malloc(sizeof(double) * n);
    for (int b = 0; b < h->nb; b++) {
        int m = h->m[b];
        combine(h, b, coef[0], coef + 1, Q0);
        for (int i = 0; i < n; i++) y[i] = sign1 * coef[(n + 1) + 1 + i];
        combine(h, b, sign1 * coef[n + 1], y, Q1);
        combine(h, b, coef[2 * (n + 1)], coef + 2 * (n + 1) + 1, Q2);
        if (h->kind[b] == ORC_DIAG) {
            for (int j = 0; j < m; j++) {
                if (!(Q0[j] > 0.0)) { *status = ORC_NOT_INTERIOR; free(y); return NAN; }
                double t = first_root_scalar(Q0[j], Q1[j], Q2[j]);
                if (t < best && t <= horizon) { best = t; *bhit = b; *jhit = j; }
            }
        } else {
            int it = 0;
            double t = curve2_dense(m, Q0, Q1, Q2, horizon, s, status, &it);
            *iters += it;
            if (*status == ORC_NOT_INTERIOR) { free(y); return NAN; }
            if (t < best) { best = t; *bhit = b; *jhit = -1; }
        }
    }
    free(y);
    return best;
}

int orc_intersect_curve2(const orc_lmi* h, int batch, const double* coef, double horizon,
                         double* tm, double* tp, int32_t* st, int32_t* iters) {
    if (!h || batch < 0 || (batch && (!coef || !tm || !tp || !st))) return ORC_EINVAL;
    scratch s;
    if (scratch_alloc(h, &s)) { scratch_free(&s); return ORC_ENOMEM; }
    size_t mm = (size_t)max_block(h);
    double* Q0 = (double*)malloc(sizeof(double) * mm * mm);
    double* Q1 = (double*)malloc(sizeof(double) * mm * mm);
    double* Q2 = (double*)malloc(sizeof(double) * mm * mm);
    int n = h->n;
    for (int e = 0; e < batch; e++) {
        const double* ce = coef + (size_t)e * 3 * (n + 1);
        int status = ORC_OK, it = 0, bh, jh;
        double p = curve2_first(h, ce, 1.0, horizon, &s, Q0, Q1, Q2, &status, &it, &bh, &jh);
        double q = NAN;
        if (status != ORC_NOT_INTERIOR)
            q = curve2_first(h, ce, -1.0, horizon, &s, Q0, Q1, Q2, &status, &it, &bh, &jh);
        tp[e] = p;
        tm[e] = (status == ORC_NOT_INTERIOR) ? NAN : -q;
        if (status == ORC_NOT_INTERIOR) tp[e] = NAN;
        st[e] = status;
        if (iters) iters[e] = it;
    }
    free(Q0); free(Q1); free(Q2);
    scratch_free(&s);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Truncated normal on a chord                                               */
/* ------------------------------------------------------------------------ */

static double upper_tail(double z) { return 0.5 * erfc(z / 1.4142135623730950488); }
static double lower_tail(double z) { return 0.5 * erfc(-z / 1.4142135623730950488); }

/* Mass of N(0,1) on [lo, z], tail-stable. */
static double mass(double lo, double z) {
    if (lo >= 0.0) return upper_tail(lo) - upper_tail(z);
    return lower_tail(z) - lower_tail(lo);
}

/* Sample z ~ N(0,1) truncated to [lo, hi] by inverting the CDF with
 * bisection (plain and monotone; stops when the bracket cannot shrink). */
static double trunc_normal(double lo, double hi, double u) {
    double total = mass(lo, hi);
    if (!(total > 0.0)) return 0.5 * (lo + hi);
    double target = u * total;
    double a = lo, b = hi;
    for (int it = 0; it < 400; it++) {
        double mid = 0.5 * (a + b);
        if (mid <= a || mid >= b) break;
        if (mass(lo, mid) < target) a = mid; else b = mid;
    }
    return 0.5 * (a + b);
}

/* Position on the chord [t-, t+] of x + t v (|v| = 1) under the target
 * restricted to the line (Alg. Hit-and-Run): uniform, or for
 * exp(-a |y|^2) the normal N(-<x,v>, 1/(2a)) truncated to the chord. */
static double chord_sample(int n, const double* x, const double* v, double vv, double tm, double tp,
                           double gauss_a, double u) {
    if (gauss_a <= 0.0) return tm + u * (tp - tm);
    double xv = 0.0;
    for (int i = 0; i < n; i++) xv += x[i] * v[i];
    double mu = -xv / vv, sig = 1.0 / sqrt(2.0 * gauss_a * vv);
    double z = trunc_normal((tm - mu) / sig, (tp - mu) / sig, u);
    double t = mu + sig * z;
    if (t < tm) t = tm;
    if (t > tp) t = tp;
    return t;
}

/* Position on the chord [t-, t+] of x + t v under the Boltzmann density
 * exp(-<c, y> / T) (the optimisation section, eq. (sdp)): along the line the
 * density is proportional to exp(-lam t), lam = <c, v> / T, a truncated
 * exponential, sampled by inverting its CDF.  For lam >= 0 the CDF from t-
 * is (1 - e^{-lam (t - t-)}) / (1 - e^{-lam L}), L = t+ - t-; for lam < 0 the
 * same form is taken from t+ backwards with 1 - u, so that t grows with u. */
static double chord_sample_boltz(int n, const double* x, const double* v, const double* c, double T,
                                 double tm, double tp, double u) {
    double cv = 0.0;
    for (int i = 0; i < n; i++) cv += c[i] * v[i];
    (void)x;
    double lam = cv / T, L = tp - tm;
    if (fabs(lam * L) < 1e-12) return tm + u * L;
    double t;
    if (lam > 0.0) {
        t = tm - log1p(u * expm1(-lam * L)) / lam;
    } else {
        double mu = -lam;
        t = tp + log1p((1.0 - u) * expm1(-mu * L)) / mu;
    }
    if (t < tm) t = tm;
    if (t > tp) t = tp;
    return t;
}

/* ------------------------------------------------------------------------ */
/* Walks                                                                     */
/* ------------------------------------------------------------------------ */

static void random_unit(uint64_t seed, uint32_t chain, uint32_t step, uint32_t tag, int n, double* v) {
    draw_normals(seed, chain, step, tag, n, v);
    double nn = 0.0;
    for (int i = 0; i < n; i++) nn += v[i] * v[i];
    nn = sqrt(nn);
    for (int i = 0; i < n; i++) v[i] /= nn;
}

/* HMC-with-reflections trajectory for exp(-|x|^2 / (2 sigma^2)):
 * the Hamiltonian ODE of eq. (ode_ham) has the exact solution
 * Phi(theta) = p cos(theta) + sigma v sin(theta), theta = t / sigma; with
 * u = tan(theta/2), (1+u^2) F(Phi) = F(p) + u 2 sigma B(v) + u^2 F(-p). */
static void hmc_rotate(int n, double sigma, double th, double* p, double* v) {
    double c = cos(th), s = sin(th);
    for (int i = 0; i < n; i++) {
        double pi = p[i], vi = v[i];
        p[i] = pi * c + sigma * vi * s;
        v[i] = -pi / sigma * s + vi * c;
    }
}

/* Kernel vector of F(p) on block b (eigenvector of its smallest eigenvalue). */
static void kernel_vector(const orc_lmi* h, int b, const double* p, scratch* s, double* u) {
    int m = h->m[b];
    combine(h, b, 1.0, p, s->C);
    jacobi(m, s->C, s->V);
    int imin = 0;
    for (int k = 1; k < m; k++)
        if (s->C[(size_t)k * m + k] < s->C[(size_t)imin * m + imin]) imin = k;
    for (int i = 0; i < m; i++) u[i] = s->V[(size_t)i * m + imin];
}

typedef struct {
    double calls, refl, caps, notint, nonsmooth, steps, noconv;
} wstats;

/* One step of each walk for one chain; x is updated in place. */
static void walk_step(const orc_lmi* h, int kind, uint64_t seed, uint32_t chain, uint32_t step,
                      double tau, int rho, double gauss_a, const double* bc, double bT, double pullback,
                      double* x, double* v, double* p, double* s_dir, double* u, double* coef, scratch* s,
                      double* Q0, double* Q1, double* Q2, wstats* ws) {
    int n = h->n;
    ws->steps += 1;
    if (kind == ORC_HNR || kind == ORC_CHNR) {
        double uu[2];
        if (kind == ORC_HNR) {
            random_unit(seed, chain, step, TAG_DIR, n, v);
        } else {
            draw_u2(seed, chain, step, 0, TAG_COORD, uu);
            int j = (int)floor(uu[0] * n);
            if (j >= n) j = n - 1;
            for (int i = 0; i < n; i++) v[i] = 0.0;
            v[j] = 1.0;
        }
        line_res r = line_oracle(h, x, v, s, NULL);
        ws->calls += 1;
        if (r.status == ORC_NOT_INTERIOR) { ws->notint += 1; return; }
        if (r.status == ORC_NOCONV) ws->noconv += 1;
        if (isinf(r.tp) || isinf(r.tm)) return; /* unbounded chord: stay */
        draw_u2(seed, chain, step, 0, TAG_POS, uu);
        /* the Boltzmann chord is sampled on [(1-pullback) t-, (1-pullback) t+]:
         * at low temperature its mass sits within T / <c, v> of an end, and a
         * point closer to the boundary than the rounding of F would stop the
         * chain (the reflections' pull-back, applied to the chord ends) */
        double t = bc ? chord_sample_boltz(n, x, v, bc, bT, (1.0 - pullback) * r.tm, (1.0 - pullback) * r.tp, uu[0])
                      : chord_sample(n, x, v, 1.0, r.tm, r.tp, gauss_a, uu[0]);
        /* every chord point at least the pull-back from the ends: a point
         * within the roots' own error of the boundary may lie outside */
        if (t < (1.0 - pullback) * r.tm) t = (1.0 - pullback) * r.tm;
        if (t > (1.0 - pullback) * r.tp) t = (1.0 - pullback) * r.tp;
        for (int i = 0; i < n; i++) x[i] += t * v[i];
        return;
    }
    double uu[2];
    draw_u2(seed, chain, step, 0, TAG_LEN, uu);
    if (kind == ORC_BILLIARD) {
        /* Alg. Billiard: ell = -tau ln eta, uniform direction, reflect until
         * ell is used up; more than rho reflections -> stay. */
        double ell = -tau * log(uu[0]);
        random_unit(seed, chain, step, TAG_DIR, n, v);
        memcpy(p, x, sizeof(double) * n);
        int nref = 0;
        for (;;) {
            line_res r = line_oracle(h, p, v, s, u);
            ws->calls += 1;
            if (r.status == ORC_NOT_INTERIOR) { ws->notint += 1; return; }
            if (r.status == ORC_NOCONV) ws->noconv += 1;
            if (r.tp >= ell) {
                /* the step ends inside: at ell, but never nearer the boundary
                 * than the pull-back of a reflection */
                double te = ell < (1.0 - pullback) * r.tp ? ell : (1.0 - pullback) * r.tp;
                for (int i = 0; i < n; i++) p[i] += te * v[i];
                break;
            }
            normal_at(h, r.bplus, r.jplus, u, s->w);
            int zero = reflect_dir(n, v, s->w, s_dir);
            if (zero || r.degenerate || r.tie) ws->nonsmooth += 1;
            for (int i = 0; i < n; i++) p[i] += (1.0 - pullback) * r.tp * v[i];
            ell -= r.tp;
            memcpy(v, s_dir, sizeof(double) * n);
            nref++;
            ws->refl += 1;
            if (nref > rho) { ws->caps += 1; return; }
        }
        memcpy(x, p, sizeof(double) * n);
        return;
    }
    if (bc) {
        /* Alg. HMC with reflections for the Boltzmann density exp(-<c, x> / T):
         * the ODE of eq. (boltz_ode) has the solution
         * p(t) = p + t v - t^2 c / (2T), velocity v - t c / T, so
         * F(p(t)) = F(p) + t B(v) + t^2 B(-c / (2T)): a degree-2 curve whose
         * first root inside the remaining travel time ends the segment. */
        double ell = tau * uu[0];
        draw_normals(seed, chain, step, TAG_MOM, n, v);
        memcpy(p, x, sizeof(double) * n);
        int nref = 0;
        while (ell > 0.0) {
            coef[0] = 1.0;
            for (int i = 0; i < n; i++) coef[1 + i] = p[i];
            coef[n + 1] = 0.0;
            for (int i = 0; i < n; i++) coef[n + 2 + i] = v[i];
            coef[2 * (n + 1)] = 0.0;
            for (int i = 0; i < n; i++) coef[2 * (n + 1) + 1 + i] = -bc[i] / (2.0 * bT);
            int status = ORC_OK, it = 0, bh, jh;
            double ts = curve2_first(h, coef, 1.0, ell, s, Q0, Q1, Q2, &status, &it, &bh, &jh);
            ws->calls += 1;
            if (status == ORC_NOT_INTERIOR) { ws->notint += 1; return; }
            if (status == ORC_NOCONV) ws->noconv += 1;
            if (isinf(ts)) {
                /* no boundary within the travel time left: fly to its end */
                for (int i = 0; i < n; i++) {
                    p[i] += ell * v[i] - ell * ell * bc[i] / (2.0 * bT);
                    v[i] -= ell * bc[i] / bT;
                }
                ell = 0.0;
                break;
            }
            /* hit point, velocity there, normal, reflected velocity */
            double* ph = s_dir;
            double* vh = s->w;
            for (int i = 0; i < n; i++) {
                ph[i] = p[i] + ts * v[i] - ts * ts * bc[i] / (2.0 * bT);
                vh[i] = v[i] - ts * bc[i] / bT;
            }
            double* wn = (double*)malloc(sizeof(double) * n);
            if (h->kind[bh] == ORC_DENSE) kernel_vector(h, bh, ph, s, u);
            normal_at(h, bh, jh, u, wn);
            double* snew = (double*)malloc(sizeof(double) * n);
            int zero = reflect_dir(n, vh, wn, snew);
            if (zero) ws->nonsmooth += 1;
            double t1 = (1.0 - pullback) * ts;
            for (int i = 0; i < n; i++) p[i] += t1 * v[i] - t1 * t1 * bc[i] / (2.0 * bT);
            memcpy(v, snew, sizeof(double) * n);
            free(wn); free(snew);
            ell -= ts;
            nref++;
            ws->refl += 1;
            if (nref > rho) { ws->caps += 1; return; }
        }
        memcpy(x, p, sizeof(double) * n);
        return;
    }
    /* Alg. HMC with reflections, Gaussian target exp(-|x|^2/(2 sigma^2)). */
    double sigma = 1.0 / sqrt(2.0 * gauss_a);
    double ell = tau * uu[0];
    draw_normals(seed, chain, step, TAG_MOM, n, v);
    memcpy(p, x, sizeof(double) * n);
    int nref = 0;
    const double half_pi = 1.5707963267948966192313216916398;
    while (ell > 0.0) {
        double th_h = ell / sigma < half_pi ? ell / sigma : half_pi;
        double u_h = tan(0.5 * th_h);
        coef[0] = 1.0;
        for (int i = 0; i < n; i++) coef[1 + i] = p[i];
        coef[n + 1] = 0.0;
        for (int i = 0; i < n; i++) coef[n + 2 + i] = 2.0 * sigma * v[i];
        coef[2 * (n + 1)] = 1.0;
        for (int i = 0; i < n; i++) coef[2 * (n + 1) + 1 + i] = -p[i];
        int status = ORC_OK, it = 0, bh, jh;
        double ustar = curve2_first(h, coef, 1.0, u_h, s, Q0, Q1, Q2, &status, &it, &bh, &jh);
        ws->calls += 1;
        if (status == ORC_NOT_INTERIOR) { ws->notint += 1; return; }
        if (status == ORC_NOCONV) ws->noconv += 1;
        if (isinf(ustar)) {
            hmc_rotate(n, sigma, th_h, p, v);
            ell -= sigma * th_h;
            continue;
        }
        double th = 2.0 * atan(ustar);
        /* hit point and velocity dPhi/dt there */
        double* ph = s_dir;
        memcpy(ph, p, sizeof(double) * n);
        double* vh = s->w; /* temporarily the velocity */
        memcpy(vh, v, sizeof(double) * n);
        hmc_rotate(n, sigma, th, ph, vh);
        double* wn = (double*)malloc(sizeof(double) * n);
        if (h->kind[bh] == ORC_DENSE) kernel_vector(h, bh, ph, s, u);
        normal_at(h, bh, jh, u, wn);
        double* snew = (double*)malloc(sizeof(double) * n);
        int zero = reflect_dir(n, vh, wn, snew);
        if (zero) ws->nonsmooth += 1;
        double* vv0 = (double*)malloc(sizeof(double) * n);
        memcpy(vv0, v, sizeof(double) * n);
        hmc_rotate(n, sigma, (1.0 - pullback) * th, p, vv0);
        memcpy(v, snew, sizeof(double) * n);
        free(wn); free(snew); free(vv0);
        ell -= sigma * th;
        nref++;
        ws->refl += 1;
        if (nref > rho) { ws->caps += 1; return; }
    }
    memcpy(x, p, sizeof(double) * n);
}

int orc_walk(const orc_lmi* h, int kind, int chains, const double* x0, int64_t steps,
             uint64_t seed, double tau, int rho, double gauss_a, double pullback,
             int thin, double* x_out, double* samples, double* stats) {
    if (!h || chains < 0 || steps < 0 || (chains && (!x0 || !x_out))) return ORC_EINVAL;
    if (kind < ORC_HNR || kind > ORC_HMC) return ORC_EINVAL;
    if (kind == ORC_HMC && !(gauss_a > 0.0)) return ORC_EINVAL;
    int n = h->n;
    scratch s;
    if (scratch_alloc(h, &s)) { scratch_free(&s); return ORC_ENOMEM; }
    size_t mm = (size_t)max_block(h);
    double* v = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* sd = (double*)malloc(sizeof(double) * n);
    double* u = (double*)malloc(sizeof(double) * mm);
    double* coef = (double*)malloc(sizeof(double) * 3 * (n + 1));
    double* Q0 = (double*)malloc(sizeof(double) * mm * mm);
    double* Q1 = (double*)malloc(sizeof(double) * mm * mm);
    double* Q2 = (double*)malloc(sizeof(double) * mm * mm);
    wstats ws = {0, 0, 0, 0, 0, 0, 0};
    int64_t nsamp = thin > 0 ? steps / thin : 0;
    for (int c = 0; c < chains; c++) {
        double* x = x_out + (size_t)c * n;
        memcpy(x, x0 + (size_t)c * n, sizeof(double) * n);
        for (int64_t k = 0; k < steps; k++) {
            walk_step(h, kind, seed, (uint32_t)c, (uint32_t)k, tau, rho, gauss_a, NULL, 0.0, pullback, x, v,
                      p, sd, u, coef, &s, Q0, Q1, Q2, &ws);
            if (samples && thin > 0 && (k + 1) % thin == 0) {
                int64_t j = (k + 1) / thin - 1;
                memcpy(samples + ((size_t)c * nsamp + j) * n, x, sizeof(double) * n);
            }
        }
    }
    if (stats) {
        stats[0] = ws.calls; stats[1] = ws.refl; stats[2] = ws.caps; stats[3] = ws.notint;
        stats[4] = ws.nonsmooth; stats[5] = ws.steps; stats[6] = ws.noconv; stats[7] = 0.0;
    }
    free(v); free(p); free(sd); free(u); free(coef); free(Q0); free(Q1); free(Q2);
    scratch_free(&s);
    return ORC_OK;
}

/* Walks on the Boltzmann density exp(-<c, x> / T) truncated to S (the
 * optimisation section): Hit-and-Run and coordinate Hit-and-Run with the
 * truncated exponential on each chord, HMC with reflections on the curve of
 * eq. (boltz_ode).  `steps` steps of chain `chain` from x_in, step k drawing
 * with counter (chain, step0 + k); every thin-th point into samples
 * (nullable); counts added to stats (8 entries, nullable). */
static int walk_chain_boltz(const orc_lmi* h, int kind, int chain, const double* x_in, int64_t step0,
                            int64_t steps, uint64_t seed, double tau, int rho, const double* c, double T,
                            double pullback, int thin, double* samples, double* x_out, double* stats) {
    int n = h->n;
    scratch s;
    if (scratch_alloc(h, &s)) { scratch_free(&s); return ORC_ENOMEM; }
    size_t mm = (size_t)max_block(h);
    double* v = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* sd = (double*)malloc(sizeof(double) * n);
    double* u = (double*)malloc(sizeof(double) * mm);
    double* coef = (double*)malloc(sizeof(double) * 3 * (n + 1));
    double* Q0 = (double*)malloc(sizeof(double) * mm * mm);
    double* Q1 = (double*)malloc(sizeof(double) * mm * mm);
    double* Q2 = (double*)malloc(sizeof(double) * mm * mm);
    wstats ws = {0, 0, 0, 0, 0, 0, 0};
    memcpy(x_out, x_in, sizeof(double) * n);
    for (int64_t k = 0; k < steps; k++) {
        walk_step(h, kind, seed, (uint32_t)chain, (uint32_t)(step0 + k), tau, rho, 0.0, c, T, pullback, x_out,
                  v, p, sd, u, coef, &s, Q0, Q1, Q2, &ws);
        if (samples && thin > 0 && (k + 1) % thin == 0)
            memcpy(samples + (size_t)((k + 1) / thin - 1) * n, x_out, sizeof(double) * n);
    }
    if (stats) {
        stats[0] += ws.calls; stats[1] += ws.refl; stats[2] += ws.caps; stats[3] += ws.notint;
        stats[4] += ws.nonsmooth; stats[5] += ws.steps; stats[6] += ws.noconv;
    }
    free(v); free(p); free(sd); free(u); free(coef); free(Q0); free(Q1); free(Q2);
    scratch_free(&s);
    return ORC_OK;
}

int orc_walk_boltz(const orc_lmi* h, int kind, int chains, const double* x0, int64_t step0, int64_t steps,
                   uint64_t seed, double tau, int rho, const double* c, double T, double pullback,
                   int thin, double* x_out, double* samples, double* stats) {
    if (!h || chains < 0 || steps < 0 || step0 < 0 || !c || !(T > 0.0) || (chains && (!x0 || !x_out)))
        return ORC_EINVAL;
    if (kind != ORC_HNR && kind != ORC_CHNR && kind != ORC_HMC) return ORC_EINVAL;
    if (kind == ORC_HMC && !(tau > 0.0)) return ORC_EINVAL;
    int n = h->n;
    int64_t nsamp = thin > 0 ? steps / thin : 0;
    if (stats) for (int k = 0; k < 8; k++) stats[k] = 0.0;
    for (int j = 0; j < chains; j++) {
        int rc = walk_chain_boltz(h, kind, j, x0 + (size_t)j * n, step0, steps, seed, tau, rho, c, T, pullback,
                                  thin, samples ? samples + (size_t)j * nsamp * n : NULL, x_out + (size_t)j * n,
                                  stats);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}

/* Simulated annealing for min <c, x> over S (eq. (sdp); the schedule of the
 * optimisation section): at iteration i the chain walks walk_len steps of the
 * Boltzmann walk at T_i = T0 (1 - cool)^i with travel-time scale
 * tau_i = tau0 sqrt(T_i / T0) (HMC; with time measured in units of sqrt(T)
 * this is HMC at temperature T with momenta N(0, T I) and a fixed travel
 * time), then the best <c, x> seen so far is updated.
 * Per chain: x_best, f_best; best[j * iters + i] is chain j's best after
 * iteration i.  The step counter runs on across iterations. */
int orc_sdp_anneal(const orc_lmi* h, int kind, int chains, const double* x0, const double* c, double T0,
                   double cool, int iters, int walk_len, uint64_t seed, double tau0, int rho, double pullback,
                   double* x_best, double* f_best, double* best) {
    if (!h || chains < 0 || iters < 0 || walk_len < 1 || !c || !(T0 > 0.0) || !(cool >= 0.0 && cool < 1.0) ||
        (chains && (!x0 || !x_best || !f_best)))
        return ORC_EINVAL;
    int n = h->n;
    double* x = (double*)malloc(sizeof(double) * n);
    double* y = (double*)malloc(sizeof(double) * n);
    int rc = ORC_OK;
    for (int j = 0; j < chains && rc == ORC_OK; j++) {
        memcpy(x, x0 + (size_t)j * n, sizeof(double) * n);
        double fb = 0.0;
        for (int i = 0; i < n; i++) fb += c[i] * x[i];
        memcpy(x_best + (size_t)j * n, x, sizeof(double) * n);
        double T = T0;
        for (int it = 0; it < iters; it++) {
            /* one chain of the walk, with its own chain index for the draws */
            rc = walk_chain_boltz(h, kind, j, x, (int64_t)it * walk_len, walk_len, seed, tau0 * sqrt(T / T0), rho, c,
                                  T, pullback, 0, NULL, y, NULL);
            if (rc != ORC_OK) break;
            memcpy(x, y, sizeof(double) * n);
            double f = 0.0;
            for (int i = 0; i < n; i++) f += c[i] * x[i];
            if (f < fb) {
                fb = f;
                memcpy(x_best + (size_t)j * n, x, sizeof(double) * n);
            }
            if (best) best[(size_t)j * iters + it] = fb;
            T *= 1.0 - cool;
        }
        f_best[j] = fb;
    }
    free(x);
    free(y);
    return rc;
}

int orc_billiard_segment(const orc_lmi* h, int batch, const double* x, const double* v,
                         const double* ell, double pullback, double* x_new, double* v_new,
                         double* ell_left, int32_t* flags) {
    if (!h || batch < 0) return ORC_EINVAL;
    int n = h->n;
    scratch s;
    if (scratch_alloc(h, &s)) { scratch_free(&s); return ORC_ENOMEM; }
    double* u = (double*)malloc(sizeof(double) * (size_t)max_block(h));
    for (int e = 0; e < batch; e++) {
        const double* xe = x + (size_t)e * n;
        const double* ve = v + (size_t)e * n;
        double* xo = x_new + (size_t)e * n;
        double* vo = v_new + (size_t)e * n;
        line_res r = line_oracle(h, xe, ve, &s, u);
        flags[2 * e] = 0;
        flags[2 * e + 1] = r.status;
        if (r.status == ORC_NOT_INTERIOR) {
            for (int i = 0; i < n; i++) { xo[i] = NAN; vo[i] = NAN; }
            ell_left[e] = NAN;
            continue;
        }
        if (r.tp >= ell[e]) {
            double te = ell[e] < (1.0 - pullback) * r.tp ? ell[e] : (1.0 - pullback) * r.tp;
            for (int i = 0; i < n; i++) { xo[i] = xe[i] + te * ve[i]; vo[i] = ve[i]; }
            ell_left[e] = 0.0;
            continue;
        }
        normal_at(h, r.bplus, r.jplus, u, s.w);
        reflect_dir(n, ve, s.w, vo);
        for (int i = 0; i < n; i++) xo[i] = xe[i] + (1.0 - pullback) * r.tp * ve[i];
        ell_left[e] = ell[e] - r.tp;
        flags[2 * e] = 1;
    }
    free(u);
    scratch_free(&s);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Volume: telescoping product over Gaussians (eq. (telegeneric))            */
/* ------------------------------------------------------------------------ */

/* CDF of Student's t with k degrees of freedom, by Simpson integration of
 * its density; the 0.975 quantile is then found by bisection. */
static double student_cdf(double t, int k) {
    /* integrate the density from 0 to t with Simpson's rule */
    double c = exp(lgamma(0.5 * (k + 1)) - lgamma(0.5 * k)) / sqrt(k * 3.14159265358979323846);
    int N = 2000;
    double hstep = t / N, acc = 0.0;
    for (int i = 0; i <= N; i++) {
        double y = i * hstep;
        double f = c * pow(1.0 + y * y / k, -0.5 * (k + 1));
        acc += f * (i == 0 || i == N ? 1.0 : (i % 2 ? 4.0 : 2.0));
    }
    return 0.5 + acc * hstep / 3.0;
}

static double student_q975(int k) {
    double lo = 0.0, hi = 100.0;
    for (int it = 0; it < 100; it++) {
        double mid = 0.5 * (lo + hi);
        if (student_cdf(mid, k) < 0.975) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

static double logsumexp_add(double acc, double v) {
    if (acc == -INFINITY) return v;
    if (v > acc) return v + log1p(exp(acc - v));
    return acc + log1p(exp(v - acc));
}

/* vol(S) = int_S f_0 * prod_i (int_S f_{i+1} / int_S f_i), with
 * f_i = exp(-a_i |x|^2), a_i geometric from a0 to a_end over the phases and
 * a final uniform f = 1; each ratio estimated by the sample mean of
 * f_{i+1}/f_i = exp((a_i - a_{i+1})|x|^2) over Hit-and-Run samples of f_i
 * restricted to S; int_S f_0 = (pi/a0)^{n/2} Pr[X in S], X ~ N(0, I/(2 a0)),
 * by exact Gaussian draws and membership.  Chains are split into n_groups
 * independent groups; the interval is mean +- t_{0.975,g-1} sd/sqrt(g) of the
 * per-group log-volumes (the confidence interval form of Table 2). */
int orc_volume(const orc_lmi* h, int phases, int spp, int chains, int walk_len, uint64_t seed,
               double a0, double a_end, int ng, double* log_vol, double* ci_lo, double* ci_hi,
               double* log_ratios) {
    if (!h || phases < 1 || spp < 1 || chains < 1 || walk_len < 1 || ng < 2 || chains % ng) return ORC_EINVAL;
    int n = h->n;
    scratch s;
    if (scratch_alloc(h, &s)) { scratch_free(&s); return ORC_ENOMEM; }
    double* X = (double*)calloc((size_t)chains * n, sizeof(double));
    double* v = (double*)malloc(sizeof(double) * n);
    double* a = (double*)malloc(sizeof(double) * (phases + 1));
    double* gl = (double*)malloc(sizeof(double) * ng * (phases + 1)); /* per-group log terms */
    for (int i = 0; i < phases; i++)
        a[i] = phases == 1 ? a0 : a0 * pow(a_end / a0, (double)i / (phases - 1));
    a[phases] = 0.0;
    int per_group = chains / ng;
    /* int_S f_0 per group by exact Gaussian draws */
    int n0 = spp;
    double sd0 = 1.0 / sqrt(2.0 * a[0]);
    for (int g = 0; g < ng; g++) {
        int hits = 0;
        for (int k = 0; k < n0; k++) {
            draw_normals(seed, (uint32_t)g, (uint32_t)k, TAG_GAUSS0, n, v);
            for (int i = 0; i < n; i++) v[i] *= sd0;
            int8_t in;
            orc_membership(h, 1, v, &in);
            hits += in;
        }
        double pr = (double)hits / n0;
        gl[g * (phases + 1)] = 0.5 * n * log(3.14159265358979323846 / a[0]) + log(pr);
    }
    int spc = (spp + chains - 1) / chains; /* samples per chain per phase */
    for (int ph = 0; ph < phases; ph++) {
        double* acc = (double*)malloc(sizeof(double) * ng);
        int* cnt = (int*)calloc(ng, sizeof(int));
        for (int g = 0; g < ng; g++) acc[g] = -INFINITY;
        for (int c = 0; c < chains; c++) {
            double* x = X + (size_t)c * n;
            int g = c / per_group;
            for (int k = 0; k < spc; k++) {
                for (int w = 0; w < walk_len; w++) {
                    uint32_t step = (uint32_t)(k * walk_len + w);
                    uint32_t tagbase = (uint32_t)(ph + 1) << 8;
                    random_unit(seed, (uint32_t)c, step, tagbase | TAG_DIR, n, v);
                    line_res r = line_oracle(h, x, v, &s, NULL);
                    if (r.status == ORC_NOT_INTERIOR || isinf(r.tp) || isinf(r.tm)) continue;
                    double uu[2];
                    draw_u2(seed, (uint32_t)c, step, 0, tagbase | TAG_POS, uu);
                    double t = chord_sample(n, x, v, 1.0, r.tm, r.tp, a[ph], uu[0]);
                    /* at least the walks' pull-back 1e-6 from the chord's ends */
                    if (t < (1.0 - 1e-6) * r.tm) t = (1.0 - 1e-6) * r.tm;
                    if (t > (1.0 - 1e-6) * r.tp) t = (1.0 - 1e-6) * r.tp;
                    for (int i = 0; i < n; i++) x[i] += t * v[i];
                }
                double r2 = 0.0;
                for (int i = 0; i < n; i++) r2 += x[i] * x[i];
                acc[g] = logsumexp_add(acc[g], (a[ph] - a[ph + 1]) * r2);
                cnt[g]++;
            }
        }
        for (int g = 0; g < ng; g++) gl[g * (phases + 1) + ph + 1] = acc[g] - log((double)cnt[g]);
        free(acc);
        free(cnt);
    }
    double mean = 0.0;
    double* lv = (double*)malloc(sizeof(double) * ng);
    for (int g = 0; g < ng; g++) {
        lv[g] = 0.0;
        for (int k = 0; k <= phases; k++) lv[g] += gl[g * (phases + 1) + k];
        mean += lv[g];
    }
    mean /= ng;
    double var = 0.0;
    for (int g = 0; g < ng; g++) var += (lv[g] - mean) * (lv[g] - mean);
    var /= (ng - 1);
    double half = student_q975(ng - 1) * sqrt(var / ng);
    *log_vol = mean;
    *ci_lo = mean - half;
    *ci_hi = mean + half;
    if (log_ratios)
        for (int k = 0; k <= phases; k++) {
            double m = 0.0;
            for (int g = 0; g < ng; g++) m += gl[g * (phases + 1) + k];
            log_ratios[k] = m / ng;
        }
    free(lv); free(X); free(v); free(a); free(gl);
    scratch_free(&s);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Volume: the ball sequence of eq. (mmc_vol)                                */
/* ------------------------------------------------------------------------ */

enum { TAG_BALL = 7, TAG_BALL_R = 8 };

/* One billiard step (Alg. Billiard) inside S cap rho B (rho = INFINITY: S):
 * the segment ends at the first of t+ of S, the ball's exit
 * -<p, v> + sqrt(<p, v>^2 + rho^2 - |p|^2) and the length left; a hit
 * reflects on S's normal or on the ball's radial normal p + t v.  More than
 * 10 n reflections: the chain stays. */
static void billiard_ball_step(const orc_lmi* h, uint64_t seed, uint32_t chain, uint32_t step, uint32_t tagbase,
                               double tau, double rho, double pullback, double* x, double* v, double* p,
                               double* sdir, double* u, double* w, scratch* s) {
    int n = h->n;
    double uu[2];
    draw_u2(seed, chain, step, 0, tagbase | TAG_LEN, uu);
    double ell = -tau * log(uu[0]);
    random_unit(seed, chain, step, tagbase | TAG_DIR, n, v);
    memcpy(p, x, sizeof(double) * n);
    int nref = 0;
    for (;;) {
        line_res r = line_oracle(h, p, v, s, u);
        if (r.status == ORC_NOT_INTERIOR) return;
        double tb = INFINITY;
        if (isfinite(rho)) {
            double pv = 0.0, pp = 0.0;
            for (int i = 0; i < n; i++) { pv += p[i] * v[i]; pp += p[i] * p[i]; }
            double disc = pv * pv + rho * rho - pp;
            tb = -pv + sqrt(disc > 0.0 ? disc : 0.0);
        }
        double th = tb < r.tp ? tb : r.tp;
        if (th >= ell) {
            double te = ell < (1.0 - pullback) * th ? ell : (1.0 - pullback) * th;
            for (int i = 0; i < n; i++) p[i] += te * v[i];
            break;
        }
        if (tb < r.tp) {
            for (int i = 0; i < n; i++) w[i] = p[i] + tb * v[i];
        } else {
            normal_at(h, r.bplus, r.jplus, u, w);
        }
        reflect_dir(n, v, w, sdir);
        for (int i = 0; i < n; i++) p[i] += (1.0 - pullback) * th * v[i];
        ell -= th;
        memcpy(v, sdir, sizeof(double) * n);
        if (++nref > 10 * n) return;
    }
    memcpy(x, p, sizeof(double) * n);
}

static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* vol(S) by the ball sequence S_i = S cap rho_i B (eq. (mmc_vol)): rho_0 =
 * infinity (S itself); in phase i every chain walks burn_in billiard steps in
 * S_i, then keeps spc samples walk_len steps apart.  The next radius
 * rho_{i+1} is the q-quantile of |x| over the first half of the samples (all
 * chains), and vol(S_{i+1}) / vol(S_i) is the fraction of the second half
 * inside rho_{i+1} B, per group of chains.  The sequence ends at the first
 * rho_k whose ball has at least a fraction q inside S by ball_draws exact
 * uniform draws per group; vol(S_k) = vol(rho_k B) times that group's
 * fraction.  Chains outside the next ball are moved radially onto
 * (1 - 1e-6) rho_{i+1} (inside S: S is convex and holds 0).  Interval: mean
 * +- t_{0.975, g-1} sd / sqrt(g) of the per-group log-volumes.  Returns
 * ORC_NOCONV if max_phases phases do not reach a ball mostly inside S. */
int orc_volume_balls(const orc_lmi* h, int chains, int spc, int walk_len, int burn_in, double q, int max_phases,
                     int ball_draws, uint64_t seed, double tau, int ng, double* log_vol, double* ci_lo,
                     double* ci_hi, double* radii, int* phases_out) {
    if (!h || chains < 1 || spc < 2 || walk_len < 1 || burn_in < 0 || !(q > 0.0 && q < 1.0) || max_phases < 1 ||
        ball_draws < 1 || !(tau > 0.0) || ng < 2 || chains % ng || !log_vol || !ci_lo || !ci_hi)
        return ORC_EINVAL;
    int n = h->n;
    scratch s;
    if (scratch_alloc(h, &s)) { scratch_free(&s); return ORC_ENOMEM; }
    size_t mm = (size_t)max_block(h);
    double* X = (double*)calloc((size_t)chains * n, sizeof(double));
    double* v = (double*)malloc(sizeof(double) * n);
    double* p = (double*)malloc(sizeof(double) * n);
    double* sd = (double*)malloc(sizeof(double) * n);
    double* w = (double*)malloc(sizeof(double) * n);
    double* u = (double*)malloc(sizeof(double) * mm);
    double* nrm = (double*)malloc(sizeof(double) * (size_t)chains * spc);
    double* first = (double*)malloc(sizeof(double) * (size_t)chains * spc);
    double* lv = (double*)calloc(ng, sizeof(double));
    int per_group = chains / ng, h1 = spc / 2;
    double rho = INFINITY;
    int rc = ORC_NOCONV, ph;
    for (ph = 0; ph < max_phases; ph++) {
        uint32_t tagbase = (uint32_t)(ph + 1) << 8;
        if (radii) radii[ph] = rho;
        for (int c = 0; c < chains; c++) {
            double* x = X + (size_t)c * n;
            int step = 0;
            for (int b = 0; b < burn_in; b++, step++)
                billiard_ball_step(h, seed, (uint32_t)c, (uint32_t)step, tagbase, tau, rho, 1e-6, x, v, p, sd, u, w,
                                   &s);
            for (int k = 0; k < spc; k++) {
                for (int t = 0; t < walk_len; t++, step++)
                    billiard_ball_step(h, seed, (uint32_t)c, (uint32_t)step, tagbase, tau, rho, 1e-6, x, v, p, sd,
                                       u, w, &s);
                double r2 = 0.0;
                for (int i = 0; i < n; i++) r2 += x[i] * x[i];
                nrm[(size_t)c * spc + k] = sqrt(r2);
            }
        }
        /* next radius from the first halves */
        int cnt1 = 0;
        for (int c = 0; c < chains; c++)
            for (int k = 0; k < h1; k++) first[cnt1++] = nrm[(size_t)c * spc + k];
        qsort(first, cnt1, sizeof(double), cmp_double);
        int qi = (int)floor(q * cnt1);
        if (qi >= cnt1) qi = cnt1 - 1;
        double rnext = first[qi];
        /* the ratio per group from the second halves */
        for (int g = 0; g < ng; g++) {
            int in = 0, tot = 0;
            for (int c = g * per_group; c < (g + 1) * per_group; c++)
                for (int k = h1; k < spc; k++, tot++) in += nrm[(size_t)c * spc + k] <= rnext;
            lv[g] -= log((double)in / tot);
        }
        /* does the ball hold a fraction q inside S? exact uniform draws */
        int hits_all = 0;
        double* pg = (double*)malloc(sizeof(double) * ng);
        for (int g = 0; g < ng; g++) {
            int hits = 0;
            for (int k = 0; k < ball_draws; k++) {
                draw_normals(seed, (uint32_t)g, (uint32_t)k, tagbase | TAG_BALL, n, v);
                double nn = 0.0;
                for (int i = 0; i < n; i++) nn += v[i] * v[i];
                double uu[2];
                draw_u2(seed, (uint32_t)g, (uint32_t)k, 0, tagbase | TAG_BALL_R, uu);
                double rad = rnext * pow(uu[0], 1.0 / n) / sqrt(nn);
                for (int i = 0; i < n; i++) v[i] *= rad;
                int8_t inside;
                orc_membership(h, 1, v, &inside);
                hits += inside;
            }
            pg[g] = (double)hits / ball_draws;
            hits_all += hits;
        }
        rho = rnext;
        if ((double)hits_all / ((double)ng * ball_draws) >= q) {
            double lball = 0.5 * n * log(3.14159265358979323846) + n * log(rho) - lgamma(0.5 * n + 1.0);
            for (int g = 0; g < ng; g++) lv[g] += lball + log(pg[g]);
            free(pg);
            if (radii) radii[ph + 1] = rho;
            rc = ORC_OK;
            ph++;
            break;
        }
        free(pg);
        /* chains into the next ball */
        for (int c = 0; c < chains; c++) {
            double* x = X + (size_t)c * n;
            double r2 = 0.0;
            for (int i = 0; i < n; i++) r2 += x[i] * x[i];
            double lim = (1.0 - 1e-6) * rho;
            if (r2 > lim * lim) {
                double sc = lim / sqrt(r2);
                for (int i = 0; i < n; i++) x[i] *= sc;
            }
        }
    }
    if (phases_out) *phases_out = ph;
    if (rc == ORC_OK) {
        double mean = 0.0, var = 0.0;
        for (int g = 0; g < ng; g++) mean += lv[g];
        mean /= ng;
        for (int g = 0; g < ng; g++) var += (lv[g] - mean) * (lv[g] - mean);
        var /= (ng - 1);
        double half = student_q975(ng - 1) * sqrt(var / ng);
        *log_vol = mean;
        *ci_lo = mean - half;
        *ci_hi = mean + half;
    }
    free(X); free(v); free(p); free(sd); free(w); free(u); free(nrm); free(first); free(lv);
    scratch_free(&s);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* MLP (the learned bracket's network), FP64                                 */
/* ------------------------------------------------------------------------ */

int64_t orc_mlp_nparams(int nl, const int* dims) {
    int64_t np = 0;
    for (int l = 0; l < nl; l++) np += (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
    return np;
}

/* exact GELU: x * Phi(x) */
static double gelu(double x) { return 0.5 * x * erfc(-x / 1.4142135623730950488); }
static double gelu_d(double x) {
    return 0.5 * erfc(-x / 1.4142135623730950488) + x * exp(-0.5 * x * x) * 0.39894228040143267794;
}

/* Forward pass keeping pre-activations Z_l and activations H_l. */
static void mlp_fwd_all(int nl, const int* dims, const double* P, int B, const double* X,
                        double** Z, double** H) {
    const double* in = X;
    const double* w = P;
    for (int l = 0; l < nl; l++) {
        int di = dims[l], dout = dims[l + 1];
        const double* bias = w + (size_t)di * dout;
        for (int r = 0; r < B; r++)
            for (int o = 0; o < dout; o++) {
                double acc = bias[o];
                for (int k = 0; k < di; k++) acc += in[(size_t)r * di + k] * w[(size_t)k * dout + o];
                Z[l][(size_t)r * dout + o] = acc;
                H[l][(size_t)r * dout + o] = (l < nl - 1) ? gelu(acc) : acc;
            }
        in = H[l];
        w = bias + dout;
    }
}

int orc_mlp_forward(int nl, const int* dims, const double* P, int B, const double* X, double* Y) {
    if (nl < 1 || B < 0) return ORC_EINVAL;
    double** Z = (double**)malloc(sizeof(double*) * nl);
    double** H = (double**)malloc(sizeof(double*) * nl);
    for (int l = 0; l < nl; l++) {
        Z[l] = (double*)malloc(sizeof(double) * (size_t)B * dims[l + 1]);
        H[l] = (double*)malloc(sizeof(double) * (size_t)B * dims[l + 1]);
    }
    mlp_fwd_all(nl, dims, P, B, X, Z, H);
    memcpy(Y, H[nl - 1], sizeof(double) * (size_t)B * dims[nl]);
    for (int l = 0; l < nl; l++) { free(Z[l]); free(H[l]); }
    free(Z); free(H);
    return ORC_OK;
}

/* Mean squared error and its gradient by backpropagation (chain rule through
 * each affine map and GELU). */
double orc_mlp_loss_grad(int nl, const int* dims, const double* P, int B, const double* X,
                         const double* T, double* G) {
    double** Z = (double**)malloc(sizeof(double*) * nl);
    double** H = (double**)malloc(sizeof(double*) * nl);
    for (int l = 0; l < nl; l++) {
        Z[l] = (double*)malloc(sizeof(double) * (size_t)B * dims[l + 1]);
        H[l] = (double*)malloc(sizeof(double) * (size_t)B * dims[l + 1]);
    }
    mlp_fwd_all(nl, dims, P, B, X, Z, H);
    int dl = dims[nl];
    double count = (double)B * dl, loss = 0.0;
    double* delta = (double*)malloc(sizeof(double) * (size_t)B * dl);
    for (size_t e = 0; e < (size_t)B * dl; e++) {
        double d = H[nl - 1][e] - T[e];
        loss += d * d;
        delta[e] = 2.0 * d / count;
    }
    /* parameter offsets */
    size_t* off = (size_t*)malloc(sizeof(size_t) * nl);
    size_t o = 0;
    for (int l = 0; l < nl; l++) { off[l] = o; o += (size_t)dims[l] * dims[l + 1] + dims[l + 1]; }
    for (int l = nl - 1; l >= 0; l--) {
        int di = dims[l], dout = dims[l + 1];
        const double* in = l == 0 ? X : H[l - 1];
        double* gw = G + off[l];
        double* gb = gw + (size_t)di * dout;
        for (int k = 0; k < di; k++)
            for (int c = 0; c < dout; c++) {
                double acc = 0.0;
                for (int r = 0; r < B; r++) acc += in[(size_t)r * di + k] * delta[(size_t)r * dout + c];
                gw[(size_t)k * dout + c] = acc;
            }
        for (int c = 0; c < dout; c++) {
            double acc = 0.0;
            for (int r = 0; r < B; r++) acc += delta[(size_t)r * dout + c];
            gb[c] = acc;
        }
        if (l > 0) {
            const double* w = P + off[l];
            double* nd = (double*)malloc(sizeof(double) * (size_t)B * di);
            for (int r = 0; r < B; r++)
                for (int k = 0; k < di; k++) {
                    double acc = 0.0;
                    for (int c = 0; c < dout; c++) acc += delta[(size_t)r * dout + c] * w[(size_t)k * dout + c];
                    nd[(size_t)r * di + k] = acc * gelu_d(Z[l - 1][(size_t)r * di + k]);
                }
            free(delta);
            delta = nd;
        }
    }
    free(delta);
    free(off);
    for (int l = 0; l < nl; l++) { free(Z[l]); free(H[l]); }
    free(Z); free(H);
    return loss / count;
}

/* Adam (Kingma & Ba, 2015) with bias correction, step counted from 1. */
void orc_adam_step(int64_t np, double* P, const double* G, double* m, double* v, int step,
                   double lr, double b1, double b2, double eps) {
    double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    for (int64_t i = 0; i < np; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * G[i];
        v[i] = b2 * v[i] + (1.0 - b2) * G[i] * G[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        P[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
