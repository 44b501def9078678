// Fused per-chain line oracle (paper: Alg. INTERSECTION for Phi(t) = x + t v,
// Lemma "PEP and S cap C"; Alg. REFLECTION, Lemma "Gradient of det F").
//
// One workgroup per chain: a steering wave plus 2m threads rounded up to
// whole waves.
//
//  1. F0 = F(x) + t0 B(v) (t0 = 0 on the plain path; the certified lower end of
//     the learned bracket otherwise) is read into LDS, packed by rows.
//  2. Blocked Cholesky F0 = L L^T and in-place triangular inverse W = L^{-1}
//     on 16x16 tiles with the FP64 matrix cores (v_mfma_f64_16x16x4f64);
//     the diagonal tiles are factored / inverted by one wave.
//  3. B(v) is held in registers: worker thread t keeps the 4 x 25 block of
//     the full symmetric B at rows 4 (t / 8).. and columns 25 (t % 8).., and
//     B a sums each row block's four partial rows over eight lanes by DPP.
//  4. Lanczos on C = W B W^T (W^T q from LDS, B a from registers, W b from
//     LDS) without reorthogonalisation; each vector entry belongs to the lane
//     that W b leaves holding that row, so c, alpha, beta and the next q are
//     formed in registers; the basis goes to HBM for the Ritz vector.  Every
//     few steps the extreme Ritz values of T_k are bracketed by
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
#include "spec_diag.h"

namespace spec {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int MAXH = 100;  // entries of B held in registers per worker thread (m <= 200)
constexpr int BR = 4, BC = 25;  // block of B per worker thread: BR rows x BC columns (8 BC = 2 MAXH)
constexpr int NCYCLES = 3;  // Lanczos cycles of at most kmax steps (restarts from the Ritz vector)

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

// Dense 16 x 16 tile in LDS with an XOR swizzle: element (i, j) at
// 16 i + (j ^ i), so that a column is spread over all banks.
__device__ __forceinline__ int sw(int i, int j) { return 16 * i + (j ^ i); }

// Packed offset of row r with rows past m read as row m - 1: a valid address
// whose (garbage) entries only reach results that are not stored.
__device__ __forceinline__ int rowb(int r, int m) {
    const int rr = r < m ? r : m - 1;
    return (rr * (rr + 1)) >> 1;
}

// Copy the lower part of diagonal tile K of the packed matrix into the dense
// tile T (identity on rows past m, zeros above the diagonal).  One wave.
__device__ __forceinline__ void tile_to_dense(const double* L, int m, int K, double* T, int lane) {
    for (int e = lane; e < 256; e += 64) {
        const int i = e >> 4, j = e & 15, r = 16 * K + i, c = 16 * K + j;
        double v = 0.0;
        if (j <= i) v = r < m ? L[pk(r, c)] : (i == j ? 1.0 : 0.0);
        T[sw(i, j)] = v;
    }
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void dense_to_tile(double* L, int m, int K, const double* T, int lane) {
    for (int e = lane; e < 256; e += 64) {
        const int i = e >> 4, j = e & 15, r = 16 * K + i;
        if (j <= i && r < m) L[pk(r, 16 * K + j)] = T[sw(i, j)];
    }
    __builtin_amdgcn_wave_barrier();
}

// Cholesky of the dense tile in place (one wave, 4 elements per lane).  Step
// j updates (i, k), j < k <= i, with the unscaled column: a_ik -= a_ij a_kj / d.
__device__ __forceinline__ bool dense_chol16(double* T, int lane) {
    for (int j = 0; j < 16; ++j) {
        const double d = T[sw(j, j)];
        if (!(d > 0.0)) return false;  // every lane read the same pivot
        const double ljj = sqrt(d), inv = 1.0 / ljj, invd = inv * inv;
        double nv0, nv1, nv2, nv3;
#define CHOL_UPD(q, out)                                                             \
    {                                                                                \
        const int e = lane + 64 * q, i = e >> 4, k = e & 15;                         \
        const double cur = T[sw(i, k)];                                              \
        double v = cur;                                                              \
        if (k > j && k <= i) v = cur - T[sw(i, j)] * T[sw(k, j)] * invd;             \
        else if (k == j && i > j) v = cur * inv;                                     \
        else if (k == j && i == j) v = ljj;                                          \
        out = v;                                                                     \
    }
        CHOL_UPD(0, nv0)
        CHOL_UPD(1, nv1)
        CHOL_UPD(2, nv2)
        CHOL_UPD(3, nv3)
#undef CHOL_UPD
        __builtin_amdgcn_wave_barrier();
#define CHOL_ST(q, val)                                  \
    {                                                    \
        const int e = lane + 64 * q, i = e >> 4, k = e & 15; \
        if (k >= j && k <= i) T[sw(i, k)] = val;         \
    }
        CHOL_ST(0, nv0)
        CHOL_ST(1, nv1)
        CHOL_ST(2, nv2)
        CHOL_ST(3, nv3)
#undef CHOL_ST
        __builtin_amdgcn_wave_barrier();
    }
    return true;
}

// In-place inverse of the lower-triangular dense tile, row by row:
// D_ic = (delta_ic - sum_{k=c..i-1} L_ik D_kc) / L_ii; four lanes per column
// share the sum.  One wave.
__device__ __forceinline__ void dense_trinv16(double* T, int lane) {
    const int c = lane & 15, p = lane >> 4;
    for (int i = 0; i < 16; ++i) {
        double s = 0.0;
        if (c < i)
            for (int k = c + p; k < i; k += 4) s += T[sw(i, k)] * T[sw(k, c)];
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        const double lii = T[sw(i, i)];
        const double val = c == i ? 1.0 / lii : -s / lii;
        __builtin_amdgcn_wave_barrier();
        if (p == 0 && c <= i) T[sw(i, c)] = val;
        __builtin_amdgcn_wave_barrier();
    }
}

// Lane k of each 16-lane row broadcast to the whole row (DPP row_newbcast).
// The 64-bit form is one v_mov_b64 with DPP (row_newbcast is the one DPP
// control that 64-bit moves take).
template <int K>
__device__ __forceinline__ double row_bcast(double v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xf, 0xf, true);
}

// 1 / sqrt(d) for a positive pivot: the hardware estimate refined by two
// Newton steps y <- y + y (1 - d y^2) / 2 (quadratic convergence from its
// ~2^-23 relative error to the rounding level); tiny or huge d take the
// correctly rounded library form.
__device__ __forceinline__ double rsqrt_newton(double d) {  // d in (1e-280, 1e280)
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double r = fma(-d * y, y, 1.0);
        y = fma(0.5 * y, r, y);
    }
    return y;
}
__device__ __forceinline__ double rsqrt_pivot(double d) {
    if (!(d > 1e-280 && d < 1e280)) return 1.0 / sqrt(d);
    return rsqrt_newton(d);
}

// Row broadcasts bc[K] = lane K's v for K = K0..15, issued back to back so that
// their latencies overlap (each feeds an independent product afterwards).
template <int K, bool = (K < 16)>
struct Bcast {
    __device__ __forceinline__ static void run(double v, double (&bc)[16]) {
        bc[K] = row_bcast<K>(v);
        Bcast<K + 1>::run(v, bc);
    }
};
template <int K>
struct Bcast<K, false> {
    __device__ __forceinline__ static void run(double, double (&)[16]) {}
};

// Unrolled steps of the diagonal-tile factorisation (column J, then J + 1..),
// each followed by the same step of the inverse of the factor, which needs
// exactly the values that step has just broadcast.  Factor: lane l holds row
// i = l & 15 in a[]; lane J keeps 1 / L_JJ in a[J] (its own diagonal entry is
// read only as that reciprocal afterwards).  Inverse, right-looking, for the
// column c = i a lane holds: W_Jc = s_J / L_JJ, then s_K -= L_KJ W_Jc for
// every K > J (s starts as the unit vector e_c), with L_KJ the broadcast bc[K]
// and 1 / L_JJ the reciprocal every lane has formed from the broadcast pivot.
template <int J>
struct DiagSteps {
    // trailing update of column K > J by column J: a_iK -= l_iJ l_KJ
    template <int K, bool = (K < 16)>
    struct Upd {
        __device__ __forceinline__ static void run(double (&a)[16], const double (&bc)[16]) {
            a[K] -= a[J] * bc[K];
            Upd<K + 1>::run(a, bc);
        }
    };
    template <int K>
    struct Upd<K, false> {
        __device__ __forceinline__ static void run(double (&)[16], const double (&)[16]) {}
    };
    // inverse update of s_K, K > J, by W_Jc
    template <int K, bool = (K < 16)>
    struct InvUpd {
        __device__ __forceinline__ static void run(const double (&bc)[16], double (&sv)[16], double w) {
            sv[K] -= bc[K] * w;
            InvUpd<K + 1>::run(bc, sv, w);
        }
    };
    template <int K>
    struct InvUpd<K, false> {
        __device__ __forceinline__ static void run(const double (&)[16], double (&)[16], double) {}
    };
    // keeps s_K, K > J, in registers at this point of the program: with the
    // empty volatile statements in program order, the updates of a step are
    // not sunk to their uses and the broadcasts of the next step are not
    // hoisted above them (which kept all the broadcasts live at once)
    template <int K, bool = (K < 16)>
    struct Pin {
        __device__ __forceinline__ static void run(double (&sv)[16]) {
            asm volatile("" : "+v"(sv[K]));
            Pin<K + 1>::run(sv);
        }
    };
    template <int K>
    struct Pin<K, false> {
        __device__ __forceinline__ static void run(double (&)[16]) {}
    };
    __device__ __forceinline__ static bool run(double (&a)[16], double (&sv)[16], double (&w)[16], int i) {
        __builtin_amdgcn_sched_barrier(0);  // one column at a time (bounds the live broadcasts)
        const double d = row_bcast<J>(a[J]);
        if (!(d > 0.0)) return false;  // the same pivot in every lane
        const double iv = rsqrt_pivot(d);
        a[J] = i == J ? iv : a[J] * iv;
        double bc[16];
        Bcast<J + 1>::run(a[J], bc);  // bc[K] = L_KJ
        __builtin_amdgcn_sched_barrier(0);
        Upd<J + 1>::run(a, bc);
        w[J] = sv[J] * iv;
        InvUpd<J + 1>::run(bc, sv, w[J]);
        Pin<J + 1>::run(sv);
        return DiagSteps<J + 1>::run(a, sv, w, i);
    }
};
template <>
struct DiagSteps<16> {
    __device__ __forceinline__ static bool run(double (&)[16], double (&)[16], double (&)[16], int) { return true; }
};

// y[K] -= s x[K] for K = K0..15
template <int K0, int K = K0, bool = (K < 16)>
struct SubScaled {
    __device__ __forceinline__ static void run(double (&y)[16], const double (&x)[16], double s) {
        y[K] = fma(-s, x[K], y[K]);
        SubScaled<K0, K + 1>::run(y, x, s);
    }
};
template <int K0, int K>
struct SubScaled<K0, K, false> {
    __device__ __forceinline__ static void run(double (&)[16], const double (&)[16], double) {}
};
template <int K0, int K = K0, bool = (K < 16)>
struct PinFrom {  // empty volatile statements on x[K0..15]: values formed before this point
    __device__ __forceinline__ static void run(double (&x)[16]) {
        asm volatile("" : "+v"(x[K]));
        PinFrom<K0, K + 1>::run(x);
    }
};
template <int K0, int K>
struct PinFrom<K0, K, false> {
    __device__ __forceinline__ static void run(double (&)[16]) {}
};

// The same factorisation and inverse without square roots on the dependency
// chain (elimination on the unscaled columns, as in L D L^T): with d_J the
// pivot and r_J = 1 / d_J, column J updates a_iK -= (a_iJ r_J) a_KJ and the
// inverse s_K -= a_KJ (s_J r_J) for K > J, where a_KJ is broadcast unscaled
// and so does not wait for r_J; L_KJ = a_KJ / sqrt(d_J) and W_Jc = s_J /
// sqrt(d_J) follow from one square root per lane after the last column (lane
// i keeps its own pivot d_i).  The chain of a column is then the pivot
// broadcast, the reciprocal (hardware estimate and two Newton steps) and the
// update of the next pivot; the rest of column J - 1's updates and column J's
// broadcasts are issued while the reciprocal is in flight.  `bad` is set when
// a pivot is not in (1e-280, 1e280) (not positive, NaN or extreme): the caller
// then repeats the tile with DiagSteps, which decides.
template <int J>
struct FastCol {
    __device__ __forceinline__ static void run(double (&a)[16], double (&sv)[16], double (&bp)[16], double mp, double tp,
                                               double& piv, bool& bad, int i) {
        __builtin_amdgcn_sched_barrier(0);
        const double d = row_bcast<J>(a[J]);  // a[J] of lane J: last updated by column J - 1's leading update
        double y = __builtin_amdgcn_rcp(d);
        bad |= !(d > 1e-280 && d < 1e280);
        piv = i == J ? d : piv;
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (J > 0) {  // the rest of column J - 1 (its update of column J was the leading one)
            SubScaled<J + 1>::run(a, bp, mp);
            SubScaled<J>::run(sv, bp, tp);
            PinFrom<J + 1>::run(a);
            PinFrom<J>::run(sv);
        }
        __builtin_amdgcn_sched_barrier(0);
        double bc[16];
        Bcast<J + 1>::run(a[J], bc);  // bc[K] = a_KJ, K > J
        PinFrom<J + 1>::run(bc);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const double e = fma(-d, y, 1.0);
            y = fma(y, e, y);
        }
        const double mJ = a[J] * y, tJ = sv[J] * y;
        if constexpr (J + 1 < 16) {
            a[J + 1] = fma(-mJ, bc[J + 1], a[J + 1]);  // leading update: the next pivot's column
            asm volatile("" : "+v"(a[J + 1]));
        }
        FastCol<J + 1>::run(a, sv, bc, mJ, tJ, piv, bad, i);
    }
};
template <>
struct FastCol<16> {
    __device__ __forceinline__ static void run(double (&)[16], double (&)[16], double (&)[16], double, double, double&,
                                               bool&, int) {}
};
// w[J] = sv[J] s_J with s_J broadcast from lane J
template <int J, bool = (J < 16)>
struct ScaleRows {
    __device__ __forceinline__ static void run(const double (&sv)[16], double (&w)[16], double s) {
        w[J] = sv[J] * row_bcast<J>(s);
        ScaleRows<J + 1>::run(sv, w, s);
    }
};
template <int J>
struct ScaleRows<J, false> {
    __device__ __forceinline__ static void run(const double (&)[16], double (&)[16], double) {}
};

// Diagonal tile K of the blocked factorisation, in registers of one wave:
// lane l holds row l & 15 of the tile (the four 16-lane rows of the wave hold
// the same data), factors it by columns with row broadcasts and forms the
// inverse of the factor alongside (lane l computes column l & 15:
// W_Ic = (delta_Ic - sum_{k<I} L_Ik W_kc) / L_II), which it stores in place
// of the tile (lower part; rows past m are the identity and are not stored).
// FastCol does the work; a tile with a pivot outside its range is repeated by
// DiagSteps (square root per column, library form for extreme pivots).
// Returns false when a pivot is not positive (every lane agrees).
__device__ __forceinline__ bool diag_factor16(double* L, int m, int K, int lane) {
    asm volatile("" : "+v"(lane));  // lane masks formed per call, not hoisted out of the tile loop
    const int i = lane & 15, r = 16 * K + i;
    const double* row = L + pk(r < m ? r : 16 * K, 16 * K);
    double a[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const double v = row[c];
        a[c] = r < m ? (c <= i ? v : 0.0) : (c == i ? 1.0 : 0.0);
    }
    double w[16], sv[16];
#pragma unroll
    for (int I = 0; I < 16; ++I) sv[I] = I == i ? 1.0 : 0.0;
    double bp[16], piv = 1.0;
    bool bad = false;
    FastCol<0>::run(a, sv, bp, 0.0, 0.0, piv, bad, i);
    if (!bad) {
        ScaleRows<0>::run(sv, w, rsqrt_newton(piv));  // piv in range: no pivot was flagged
    } else {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const double v = row[c];
            a[c] = r < m ? (c <= i ? v : 0.0) : (c == i ? 1.0 : 0.0);
        }
#pragma unroll
        for (int I = 0; I < 16; ++I) sv[I] = I == i ? 1.0 : 0.0;
        if (!DiagSteps<0>::run(a, sv, w, i)) return false;
    }
    if (lane < 16) {
#pragma unroll
        for (int I = 0; I < 16; ++I)
            if (I >= i && 16 * K + I < m) L[pk(16 * K + I, 16 * K) + i] = w[I];
    }
    return true;
}

// Tile (I, J), J < I, of the inverse W = L^{-1} by rows:
// W_IJ = -W_II sum_{K=J..I-1} L_IK W_KJ, with row I of L, the rows K < I of W
// (W_JJ the diagonal tile, lower part) and W_II in place.  Returned in the
// accumulator layout (lane l: rows (l >> 4) + 4 r, column l & 15), which is
// also the right-operand layout of the second product.  Rows of tile row I
// past m read row m - 1 (finite; their results are never stored).
__device__ __forceinline__ d4 inv_row_tile(const double* L, int m, int I, int J, int lane) {
    const int li = lane & 15, lh = lane >> 4;
    const double* pa = L + rowb(16 * I + li, m) + lh;  // L_IK[li][4 s + lh] at 16 K + 4 s
    d4 acc{0.0, 0.0, 0.0, 0.0};
    for (int K = J; K < I; ++K) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kr = 16 * K + 4 * s + lh;  // < m: K <= T - 2
            const double b = L[rowb(kr, m) + 16 * J + li];
            const double bv = (K > J || li <= 4 * s + lh) ? b : 0.0;  // W_JJ: lower part
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[16 * K + 4 * s], bv, acc, 0, 0, 0);
        }
    }
    const double* pw = L + rowb(16 * I + li, m) + 16 * I + lh;  // W_II[li][4 s + lh]
    d4 out{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double a = 4 * s + lh <= li ? pw[4 * s] : 0.0;
        out = __builtin_amdgcn_mfma_f64_16x16x4f64(a, acc[s], out, 0, 0, 0);
    }
    return -out;
}
__device__ __forceinline__ void store_tile(double* L, int m, int I, int J, d4 v, int lane) {
    const int li = lane & 15, lh = lane >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * I + lh + 4 * r;
        if (row < m) L[rowb(row, m) + 16 * J + li] = v[r];
    }
}

// L[e] = F[e] + sh B[e] for e < P (B null: F alone) by the bd threads of the
// block, each with 8 loads per array issued before their first use, so that
// a thread's reads from global memory are in flight together rather than one
// round trip at a time.
__device__ __forceinline__ void fill_pencil(double* L, const double* F, const double* B, double sh, int P, int t,
                                            int bd) {
    constexpr int U = 8;
    for (int e0 = t; e0 < P; e0 += U * bd) {
        double f[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * bd;
            f[u] = e < P ? F[e] : 0.0;
            b[u] = B && e < P ? B[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * bd;
            if (e < P) L[e] = B ? fma(sh, b[u], f[u]) : f[u];
        }
    }
}

// The same with F carried over from the previous round of a walk:
// F[e] = Fp[e] + s Bp[e] is written to Fo and L[e] = F[e] + sh B[e] (B null:
// F alone).  Each thread reads back nothing it wrote, so the fill can be
// repeated (another origin) without a fence.
__device__ __forceinline__ void fill_pencil_upd(double* L, const double* Fp, const double* Bp, double s, double* Fo,
                                                const double* B, double sh, int P, int t, int bd) {
    constexpr int U = 8;
    for (int e0 = t; e0 < P; e0 += U * bd) {
        double f[U], bp[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * bd;
            f[u] = e < P ? Fp[e] : 0.0;
            bp[u] = e < P ? Bp[e] : 0.0;
            b[u] = B && e < P ? B[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * bd;
            if (e < P) {
                const double fx = fma(s, bp[u], f[u]);
                Fo[e] = fx;
                L[e] = B ? fma(sh, b[u], fx) : fx;
            }
        }
    }
}

// L[e] = Q0[e] + tau (sg Q1[e] + tau Q2[e]) for e < P, loads batched as in
// fill_pencil.
__device__ __forceinline__ void fill_quadratic(double* L, const double* Q0, const double* Q1, const double* Q2,
                                               double tau, double sg, int P, int t, int bd) {
    constexpr int U = 8;
    for (int e0 = t; e0 < P; e0 += U * bd) {
        double q0[U], q1[U], q2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * bd;
            q0[u] = e < P ? Q0[e] : 0.0;
            q1[u] = e < P ? Q1[e] : 0.0;
            q2[u] = e < P ? Q2[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * bd;
            if (e < P) L[e] = q0[u] + tau * (sg * q1[u] + tau * q2[u]);
        }
    }
}

#ifndef CHOL_RHO_X2
#define CHOL_RHO_X2 4  // twice the cost of a trailing tile in inverse product steps
#endif

// Blocked Cholesky in LDS.  Returns false if F0 is not positive definite.
// It also forms the inverse W = L^{-1} by rows, row I in the trailing phase
// of step I on the waves that would otherwise wait for the next diagonal
// tile (row I of L is final after the panel of column I - 1, W_II after the
// previous trailing phase), kept in registers and stored in the next panel
// phase, when no update reads row I of L any more.  On success the tile rows
// I <= T - 2 hold W; tri_inverse forms the last one.
// `flag` is an LDS int; `D` 256 doubles of LDS scratch.
// prof (nullable): each thread adds the cycles of the diagonal-tile, panel and
// trailing-update stages to prof[0..2] and its wave's busy cycles in the
// trailing phases (up to its barrier arrival) to prof[3].
__device__ __forceinline__ bool chol_blocked(double* L, int m, double* D, int* flag, long long* prof = nullptr) {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));  // per-call lane addressing (see lanczos_extreme)
    const int lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
    const int li = lane & 15, lh = lane >> 4;
    const int T = (m + 15) / 16;
    long long c0 = 0, c1 = 0, c2 = 0, cb = 0, tc = prof ? clock64() : 0;
#define CHOL_TICK(acc)                       \
    if (prof) {                              \
        const long long tn = clock64();      \
        acc += tn - tc;                      \
        tc = tn;                             \
    }
    // A_IJ -= L_IK L_JK^T for one tile, K < J <= I
    auto trail_tile = [&](int K, int I, int J) {
        const double* pa = L + rowb(16 * I + li, m) + 16 * K + lh;
        const double* pb = L + rowb(16 * J + li, m) + 16 * K + lh;
        int ab[4];
        d4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            ab[r] = rowb(16 * I + lh + 4 * r, m) + 16 * J + li;
            acc[r] = L[ab[r]];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-pa[4 * s], pb[4 * s], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * I + lh + 4 * r, col = 16 * J + li;
            if (row < m && col <= row) L[ab[r]] = acc[r];
        }
    };
    if (wv == 0) {
        const bool ok = diag_factor16(L, m, 0, lane);
        if (lane == 0) *flag = ok ? 1 : 0;
    }
    lds_barrier();
    CHOL_TICK(c0)
    // row wrow of W computed in the last trailing phase by waves 1.. (tiles
    // j1 = wv - 1 and j2 = 2 (nw - 1) - wv, paired by size), not yet stored
    int wrow = 0;
    d4 wt1{0.0, 0.0, 0.0, 0.0}, wt2{0.0, 0.0, 0.0, 0.0};
    const int j1 = wv - 1, j2 = 2 * (nw - 1) - wv;
    auto store_wrow = [&]() {
        if (wv >= 1 && wrow >= 1) {
            if (j1 < wrow) store_tile(L, m, wrow, j1, wt1, lane);
            if (j2 < wrow) store_tile(L, m, wrow, j2, wt2, lane);
        }
    };
    for (int K = 0; K < T; ++K) {
        if (*flag == 0) return false;
        if (K + 1 == T) break;
        store_wrow();  // row K - 1 of W (no update of this step reads it)
        // panel: L_IK = A_IK W_KK^T (W_KK = L_KK^{-1}, now in the diagonal tile).
        // MFMA operands: lane l holds X[l & 15][4 s + (l >> 4)] of the left and
        // Y[l & 15][4 s + (l >> 4)] of the right factor of X Y^T; results land
        // in rows (l >> 4) + 4 r, column l & 15.
        {
            double wk[4];
            {
                const double* pw = L + rowb(16 * K + li, m) + 16 * K + lh;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const double w = pw[4 * s];
                    wk[s] = 4 * s + lh <= li ? w : 0.0;
                }
            }
            for (int I = K + 1 + wv; I < T; I += nw) {
                const double* pa = L + rowb(16 * I + li, m) + 16 * K + lh;
                d4 acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[4 * s], wk[s], acc, 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * I + lh + 4 * r;
                    if (row < m) L[rowb(row, m) + 16 * K + li] = acc[r];
                }
            }
        }
        lds_barrier();
        CHOL_TICK(c1)
        // trailing update, K < J <= I, with look-ahead: wave 0 updates the next
        // diagonal tile and factors it (its own LDS writes are seen by its later
        // reads) while the other waves update the remaining tiles
        const int R = T - K - 1;
        const long long tb = prof ? clock64() : 0;
        if (wv == 0) {
            trail_tile(K, K + 1, K + 1);
            const bool ok = diag_factor16(L, m, K + 1, lane);
            if (lane == 0) *flag = ok ? 1 : 0;
        } else {
            // tiles e = 1..N of the trailing triangle (row-major; e = 0 is wave 0's),
            // dealt in contiguous runs so that each worker's run plus its inverse
            // chains below comes out even, a tile counting CHOL_RHO_X2 / 2 product
            // steps of a chain (water level over the workers, integer arithmetic on
            // scalar registers)
            const int N = R * (R + 1) / 2 - 1;
            if (N > 0) {
                const int ws = __builtin_amdgcn_readfirstlane(wv), nwk = nw - 1;
                auto chains = [&](int v) { return max(K - (v - 1), 0) + max(K - (2 * (nw - 1) - v), 0); };
                int suml = 0;
                for (int v = 1; v < nw; ++v) suml += chains(v);
                const int lvl = 2 * suml + CHOL_RHO_X2 * N;
                int pre = 0, tot = 0, own = 0;
                for (int v = 1; v < nw; ++v) {
                    const int cap = max(lvl - 2 * nwk * chains(v), 0);
                    pre += v < ws ? cap : 0;
                    own = v == ws ? cap : own;
                    tot += cap;
                }
                const int e0 = 1 + N * pre / tot, e1 = 1 + N * (pre + own) / tot;
                int ii = 0;
                while ((ii + 1) * (ii + 2) / 2 <= e0) ++ii;
                int jj = e0 - ii * (ii + 1) / 2;
                for (int e = e0; e < e1; ++e) {
                    trail_tile(K, K + 1 + ii, K + 1 + jj);
                    if (++jj > ii) {
                        ++ii;
                        jj = 0;
                    }
                }
            }
            // row K of W (these waves would otherwise wait for the diagonal factor)
            wrow = K;
            if (j1 < K) wt1 = inv_row_tile(L, m, K, j1, lane);
            if (j2 < K) wt2 = inv_row_tile(L, m, K, j2, lane);
        }
        if (prof) cb += clock64() - tb;
        lds_barrier();
        CHOL_TICK(c2)
    }
    store_wrow();  // row T - 2 of W
    lds_barrier();
#undef CHOL_TICK
    if (prof) {
        prof[0] += c0;
        prof[1] += c1;
        prof[2] += c2;
        prof[3] += cb;
    }
    return true;
}

// Last tile row of the inverse W = L^{-1} (chol_blocked has formed the rows
// above it in place): W_T-1,J for J < T - 1 over all waves, paired by size,
// then stored once every wave has read row T - 1 of L.
// prof (nullable): thread 0 adds the cycles of its products and stores to
// prof[1], prof[2].
__device__ __forceinline__ void tri_inverse(double* L, int m, double* D, long long* prof = nullptr) {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));  // per-call lane addressing (see lanczos_extreme)
    const int lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
    const int T = (m + 15) / 16;
    long long tc = prof ? clock64() : 0, c1 = 0, c2 = 0;
    (void)D;
    if (T >= 2) {
        const int I = T - 1, ja = wv, jb = 2 * nw - 1 - wv;
        d4 va{0.0, 0.0, 0.0, 0.0}, vb{0.0, 0.0, 0.0, 0.0};
        if (ja < I) va = inv_row_tile(L, m, I, ja, lane);
        if (jb < I) vb = inv_row_tile(L, m, I, jb, lane);
        lds_barrier();
        if (prof) {
            const long long tn = clock64();
            c1 = tn - tc;
            tc = tn;
        }
        if (ja < I) store_tile(L, m, I, ja, va, lane);
        if (jb < I) store_tile(L, m, I, jb, vb, lane);
        lds_barrier();
        if (prof) c2 = clock64() - tc;
    }
    if (prof && t == 0) {
        prof[1] += c1;
        prof[2] += c2;
    }
}

// Sturm count of the k x k tridiagonal (al, be) below x: sign changes of the
// leading principal minors p_i(x) = (al_i - x) p_{i-1} - be_i^2 p_{i-2},
// rescaled so that no division is needed.
__device__ inline int sturm(const double* al, const double* be, int k, double x) {
    int cnt = 0;
    double pm = 1.0, pc = al[0] - x;  // p_{i-1}, p_i
    bool neg_prev = false;
    bool neg = pc < 0.0 || (pc == 0.0 && !neg_prev);
    cnt += neg != neg_prev;
    neg_prev = neg;
    for (int i = 1; i < k; ++i) {
        const double pn = (al[i] - x) * pc - be[i] * be[i] * pm;
        pm = pc;
        pc = pn;
        const double mag = fabs(pc);
        if (mag > 1e150 || (mag < 1e-150 && mag > 0.0)) {
            const double sc = mag > 1e150 ? 1e-150 : 1e150;
            pc *= sc;
            pm *= sc;
        }
        neg = pc < 0.0 || (pc == 0.0 && !neg_prev);
        cnt += neg != neg_prev;
        neg_prev = neg;
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

// The steering wave keeps T_k in registers: lane i holds (al_i, be_i) in A
// for i < 64 and in B for 64 <= i < 128; the recurrences read them back with
// readlane (a scalar read, no LDS round trip).
__device__ __forceinline__ double rl(double v, int i) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), i);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), i);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double tri_at(double vA, double vB, int i) { return i < 64 ? rl(vA, i) : rl(vB, i - 64); }

// Sturm count (leading-minor recurrence p_i = (al_i - x) p_{i-1} - be_i^2
// p_{i-2}, no division) on register T_k; b2 holds be_i^2.  The pair
// (p_{i-1}, p_i) is rescaled by a power of two every 8 steps.  Exact zeros
// count as positive (a measure-zero event for a multisection point).
__device__ inline int sturm_reg(double aA, double aB, double b2A, double b2B, int k, double x) {
    double pm = 1.0, pc = rl(aA, 0) - x;
    int cnt = pc < 0.0;
    // rows 1..63 live in the A registers, rows 64.. in the B registers: two
    // loops, so that no per-step select between them is needed
#define STURM_STEP(av, b2v)                                \
    {                                                      \
        const double pn = ((av) - x) * pc - (b2v) * pm;    \
        cnt += (pn < 0.0) != (pc < 0.0);                   \
        pm = pc;                                           \
        pc = pn;                                           \
        if ((i & 7) == 0) {                                \
            const int e = ilogb(fabs(pc) + fabs(pm) + 1e-300); \
            pc = ldexp(pc, -e);                            \
            pm = ldexp(pm, -e);                            \
        }                                                  \
    }
    const int k1 = k < 64 ? k : 64;
    for (int i = 1; i < k1; ++i) STURM_STEP(rl(aA, i), rl(b2A, i))
    for (int i = 64; i < k; ++i) STURM_STEP(rl(aB, i - 64), rl(b2B, i - 64))
#undef STURM_STEP
    return cnt;
}

// 1/|y| for the eigenvector y of T_k (backward recurrence, y_{k-1} = 1);
// rbA/rbB hold 1/be_i.
// Sturm count of T_k below this lane's x with T_k read from LDS (al, be; the
// same address in every lane, a broadcast): blocks of 8 steps whose loads are
// issued ahead of the recurrence, with a power-of-two rescaling after each
// block (exact, so the count is that of the plain recurrence).
__device__ inline int sturm_lds(const double* al, const double* be, int k, double x) {
    k = __builtin_amdgcn_readfirstlane(k);
    double pm = 1.0, pc = al[0] - x;
    int cnt = pc < 0.0;
#define STURM_STEP(av, bv)                                 \
    {                                                      \
        const double pn = ((av) - x) * pc - ((bv) * (bv)) * pm; \
        cnt += (pn < 0.0) != (pc < 0.0);                   \
        pm = pc;                                           \
        pc = pn;                                           \
    }
    int i = 1;
    for (; i + 8 <= k; i += 8) {
        double av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            av[u] = al[i + u];
            bv[u] = be[i + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) STURM_STEP(av[u], bv[u])
        const int e = ilogb(fabs(pc) + fabs(pm) + 1e-300);
        pc = ldexp(pc, -e);
        pm = ldexp(pm, -e);
    }
    for (; i < k; ++i) STURM_STEP(al[i], be[i])
#undef STURM_STEP
    return cnt;
}

// |s_k| of the eigenvector s of T_k for this lane's theta (normalised, last
// component), from the backward recurrence
//   y_{i-1} = ((theta - alpha_i) y_i - beta_{i+1} y_{i+1}) / beta_i,
// y_{k-1} = 1, with T_k read from LDS (a broadcast) and 1/beta_i from the
// hardware reciprocal with one Newton step (a stopping bound needs no more).
// y is rescaled every 4 steps once ss > 1e150; should ss still overflow (a run
// of tiny beta_i), the result is NaN, which no stop test accepts, rather than
// the 0 that 1/sqrt(inf) would give.
__device__ inline double backward_norm_lds(const double* al, const double* be, int k, double th) {
    k = __builtin_amdgcn_readfirstlane(k);
    double y1 = 1.0, y0 = 0.0, ss = 1.0, bn = 0.0;
    int i = k - 1;
    auto step = [&]() {
        const double ai = al[i], bi = be[i];
        double r = __builtin_amdgcn_rcp(bi);
        r = fma(r, fma(-bi, r, 1.0), r);
        r = bi != 0.0 ? r : 0.0;
        const double ym = ((th - ai) * y1 - bn * y0) * r;
        y0 = y1;
        y1 = ym;
        ss = fma(ym, ym, ss);
        bn = bi;
        --i;
    };
    for (; i >= 4; ) {
        step();
        step();
        step();
        step();
        if (ss > 1e150) {
            y0 *= 1e-75;
            y1 *= 1e-75;
            ss *= 1e-150;
        }
    }
    while (i >= 1) step();
    return ss < INFINITY ? 1.0 / sqrt(ss) : NAN;
}

__device__ inline double backward_norm_reg(double aA, double aB, double bA, double bB, double rbA, double rbB, int k,
                                           double th) {
    double y1 = 1.0, y0 = 0.0, ss = 1.0;
    for (int i = k - 1; i >= 1; --i) {
        const double ai = tri_at(aA, aB, i), rbi = tri_at(rbA, rbB, i);
        const double bn = i + 1 < k ? tri_at(bA, bB, i + 1) : 0.0;
        const double ym = ((th - ai) * y1 - bn * y0) * rbi;
        y0 = y1;
        y1 = ym;
        ss += ym * ym;
        if (ss > 1e280) {
            const double sc = 1e-140;
            y0 *= sc;
            y1 *= sc;
            ss *= sc * sc;
        }
    }
    return 1.0 / sqrt(ss);
}

// Row r of the Ritz vector z = sum_i y_i q_i of T_k for the Ritz value th,
// with y from the backward three-term recurrence (y_{k-1} = 1) and the
// stored basis rows Qg[i m + r]; normalised in y.  The rows are read from
// global memory 8 at a time ahead of the recurrence (which runs in the same
// order either way), so that their loads are in flight together.
__device__ inline double ritz_row(const double* al, const double* be, int k, double th, const double* Qg, int m,
                                  int r) {
    constexpr int U = 8;
    double zr = 0.0, y1 = 1.0, y0 = 0.0, ss = 0.0;
    for (int i0 = k - 1; i0 >= 0; i0 -= U) {
        double qv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) qv[u] = i0 - u >= 0 ? Qg[(size_t)(i0 - u) * m + r] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 - u;
            if (i < 0) break;
            zr += y1 * qv[u];
            ss += y1 * y1;
            if (i >= 1) {
                const double ym = ((th - al[i]) * y1 - (i + 1 < k ? be[i + 1] * y0 : 0.0)) / be[i];
                y0 = y1;
                y1 = ym;
            }
            if (ss > 1e280) {
                const double sc = 1e-140;
                y0 *= sc;
                y1 *= sc;
                ss *= sc * sc;
                zr *= sc;
            }
        }
    }
    return zr * (1.0 / sqrt(ss));
}

// Column c of W^T x restricted to half h of the rows [R0, m) of the wave's
// band: sum over rows rr >= c of W[rr][c] x[rr].  Rows are walked in step by
// all lanes of the wave so that they read consecutive addresses of one row.
__device__ __forceinline__ double wt_column(const double* L, const double* x, int c, int R0, int m, int h) {
    const int mid = (R0 + m) >> 1;
    const int rb = h == 0 ? R0 : mid, re = h == 0 ? mid : m;
    double s0 = 0.0, s1 = 0.0;
    int base = pk(rb, c);
    int rr = rb;
    for (; rr + 1 < re; rr += 2) {
        const double w0 = L[base], w1 = L[base + rr + 1];
        s0 += (rr >= c ? w0 : 0.0) * x[rr];
        s1 += (rr + 1 >= c ? w1 : 0.0) * x[rr + 1];
        base += 2 * rr + 3;
    }
    if (rr < re) s0 += (rr >= c ? L[base] : 0.0) * x[rr];
    return s0 + s1;
}

// Half h of row r of W x: sum over k <= r of W[r][k] x[k].
__device__ __forceinline__ double w_row(const double* L, const double* x, int r, int h) {
    const int half = (r + 2) >> 1;
    const int kb = h == 0 ? 0 : half, ke = h == 0 ? half : r + 1;
    const double* row = L + pk(r, 0);
    double s0 = 0.0, s1 = 0.0;
    int kk = kb;
    for (; kk + 1 < ke; kk += 2) {
        s0 += row[kk] * x[kk];
        s1 += row[kk + 1] * x[kk + 1];
    }
    if (kk < ke) s0 += row[kk] * x[kk];
    return s0 + s1;
}

// Balanced triangular products of the Lanczos step on the packed lower W in
// LDS, by 16 x 16 tiles.  Worker wave g takes tile columns (W^T x) or tile
// rows (W x) g and T-1-g, T tiles per side: T+1 tiles per wave (the middle
// one alone when T is odd), against 2T for the first or last band of a
// row/column split.  In a tile, lane l holds rows (l >> 4) + 4 s, s < 4, of
// column l & 15, so that one load reads 16 consecutive entries of 4 rows.

// Rows of a tile row past m are read as row m-1 (valid entries of W for every
// column left of the diagonal tile) against x = 0, so only the diagonal
// tile needs a mask; a diagonal entry right of the diagonal is replaced by 0
// before use (its address is still inside the LDS allocation: at most 15
// entries past the factor, where the scratch area lies).
// Lane moves within rows of 16 lanes by DPP (no index registers, no LDS):
// quad_perm [1,0,3,2] (lane ^ 1), [2,3,0,1] (lane ^ 2), row_ror:8
// (lane ^ 8), row_half_mirror (lane ^ 7 within 8) and row_mirror (lane ^ 15).
constexpr int DPP_X1 = 0xB1, DPP_X2 = 0x4E, DPP_X8 = 0x128, DPP_HMIR = 0x141, DPP_MIR = 0x140;
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the wave: within rows by DPP, then the four row totals.
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_mov<DPP_X1>(v);
    v += dpp_mov<DPP_X2>(v);
    v += dpp_mov<DPP_HMIR>(v);
    v += dpp_mov<DPP_MIR>(v);
    const long long b = __double_as_longlong(v);
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 16 * r);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * r);
        s += __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    return s;
}

// Minimum and maximum over the wave by the same DPP steps (no lane-address
// registers, unlike shuffles), the four row results read from lanes 0, 16, 32, 48.
template <bool MAX>
__device__ __forceinline__ double wave_ext_dpp(double v) {
    auto op = [](double x, double y) { return MAX ? fmax(x, y) : fmin(x, y); };
    v = op(v, dpp_mov<DPP_X1>(v));
    v = op(v, dpp_mov<DPP_X2>(v));
    v = op(v, dpp_mov<DPP_HMIR>(v));
    v = op(v, dpp_mov<DPP_MIR>(v));
    const long long b = __double_as_longlong(v);
    double s = v;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 16 * r);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * r);
        const double x = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
        s = r == 0 ? x : op(s, x);
    }
    return s;
}

// block_sum_lds with the wave sums by DPP (same barriers).
__device__ __forceinline__ double block_sum_dpp(double v, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum_dpp(v);
    lds_barrier();
    if (lane == 0) red[wid] = v;
    lds_barrier();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// Column sums of W^T x over tile column J (tiles I = J..T-1).  Lane l takes
// column 16 J + (l >> 2) and rows 4 q + (l & 3) of each tile (one load still
// reads 16 consecutive entries of 4 rows); the four lanes of a quad, which
// share the column, return its sum.  The byte addresses step by
// pk(r + 16) - pk(r) = 16 r + 136 entries from the diagonal tile on (which
// masks the entries right of the diagonal); in a last tile row that ends past
// m the rows past m read row m - 1 against x = 0.
__device__ __forceinline__ double wt_col(const double* L, const double* x, int m, int T, int J, int lane) {
    asm volatile("" : "+v"(lane));  // addressing formed per call, not kept live across the step loop
    const int p = lane & 3, c = 16 * J + (lane >> 2);
    const int Iend = (m & 15) ? T - 1 : T;  // tile rows with all 16 rows below m
    double s = 0.0;
    auto edge = [&](int I) {
        double w[4], xs[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * I + 4 * q + p, rr = r < m ? r : m - 1;
            xs[q] = x[rr];
            w[q] = L[pk(rr, 0) + c];
        }
        __builtin_amdgcn_sched_barrier(0);  // the loads in flight together
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * I + 4 * q + p;
            s += (r < m && c <= r ? w[q] : 0.0) * (r < m ? xs[q] : 0.0);
        }
    };
    if (J < Iend) {
        // from the diagonal tile on: incremental row bases; the diagonal tile
        // masks the entries right of the diagonal (their addresses stay inside
        // the allocation: at most 15 entries past the factor)
        const char* Lb = (const char*)L;
        const char* xb = (const char*)(x + 16 * J + p);
        int ab[4], d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * J + 4 * q + p;
            ab[q] = 8 * (pk(r, 0) + c);
            d[q] = 8 * (16 * r + 136);
        }
        {
            double w[4], xs[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                w[q] = *(const double*)(Lb + ab[q]);
                xs[q] = *(const double*)(xb + 32 * q);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                s += (c <= 16 * J + 4 * q + p ? w[q] : 0.0) * xs[q];
                ab[q] += d[q];
                d[q] += 8 * 256;
            }
            xb += 128;
        }
        for (int I = J + 1; I < Iend; ++I) {
            double w[4], xs[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                w[q] = *(const double*)(Lb + ab[q]);
                xs[q] = *(const double*)(xb + 32 * q);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                s += w[q] * xs[q];
                ab[q] += d[q];
                d[q] += 8 * 256;
            }
            xb += 128;
        }
        if (Iend < T) {
            // the last tile row ends past m: its rows past m read row m - 1 (a
            // valid, finite entry, since c < 16 (T - 1) <= m - 1 here) against x = 0
            const int abmax = 8 * (pk(m - 1, 0) + c);
            double w[4], xs[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int a = ab[q] < abmax ? ab[q] : abmax;
                w[q] = *(const double*)(Lb + a);
                xs[q] = *(const double*)(xb + 32 * q);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) s += w[q] * (16 * (T - 1) + 4 * q + p < m ? xs[q] : 0.0);
        }
    } else {
        edge(J);  // the last tile row, ending past m, is the diagonal tile
    }
    s += dpp_mov<DPP_X1>(s);
    s += dpp_mov<DPP_X2>(s);
    return s;
}

// Sum over each group of eight lanes of four per-lane accumulators, half of
// them exchanged at the first two levels (the mirrored partner within the
// eight, which differs in bit 2, then lane ^ 2): lane l ends with the total
// of a[s], s = 2 ((l >> 2) & 1) + ((l >> 1) & 1), as does lane l ^ 1.
__device__ __forceinline__ double red8x4(const double a[4], int lane) {
    const bool b2 = lane & 4, b1 = lane & 2;
    const double k0 = b2 ? a[2] : a[0], k1 = b2 ? a[3] : a[1];
    const double s0 = b2 ? a[0] : a[2], s1 = b2 ? a[1] : a[3];
    const double u0 = k0 + dpp_mov<DPP_HMIR>(s0), u1 = k1 + dpp_mov<DPP_HMIR>(s1);
    double v = (b1 ? u1 : u0) + dpp_mov<DPP_X2>(b1 ? u0 : u1);
    v += dpp_mov<DPP_X1>(v);
    return v;
}

// Sum over the 16 lanes of each lane row of four per-row accumulators,
// exchanging half of them at each of the first two levels (lane ^ 8, then
// the mirror partner within 8, which differs in bit 2): lane l ends with the
// total of a[s], s = 2 ((l >> 3) & 1) + ((l >> 2) & 1).
__device__ __forceinline__ double red16x4(const double a[4], int lane) {
    const bool b3 = lane & 8, b2 = lane & 4;
    const double k0 = b3 ? a[2] : a[0], k1 = b3 ? a[3] : a[1];
    const double s0 = b3 ? a[0] : a[2], s1 = b3 ? a[1] : a[3];
    const double u0 = k0 + dpp_mov<DPP_X8>(s0), u1 = k1 + dpp_mov<DPP_X8>(s1);
    double v = (b2 ? u1 : u0) + dpp_mov<DPP_HMIR>(b2 ? u0 : u1);
    v += dpp_mov<DPP_X2>(v);
    v += dpp_mov<DPP_X1>(v);
    return v;
}

// Row of W x that red16x4 leaves in lane l, within its tile row.
__device__ __forceinline__ int w_tiles_row(int lane) {
    return (lane >> 4) + 4 * (2 * ((lane >> 3) & 1) + ((lane >> 2) & 1));
}

// Row sums of W x over tile row I (tiles J = 0..I): lane l returns the sum
// of row 16 I + w_tiles_row(l).  The tiles left of the diagonal are read at
// fixed offsets from four row bases.
__device__ __forceinline__ double w_strip(const double* L, const double* x, int m, int I, int lane) {
    asm volatile("" : "+v"(lane));  // addressing formed per call (as in wt_col)
    const int i0 = lane >> 4, j = lane & 15;
    const double* rp[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = 16 * I + i0 + 4 * q;
        rp[q] = L + pk(r < m ? r : m - 1, 0) + j;
    }
    const double* xp = x + j;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int J = 0; J < I; ++J) {
        const double xv = xp[16 * J];
        double w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = rp[q][16 * J];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] += w[q] * xv;
    }
    {  // diagonal tile: its five loads issued together, then masked
        const int c = 16 * I + j;
        const double xr = x[c < m ? c : 0];
        double w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = rp[q][16 * I];
        __builtin_amdgcn_sched_barrier(0);
        const double xv = c < m ? xr : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] += (c <= 16 * I + i0 + 4 * q ? w[q] : 0.0) * xv;
    }
    return red16x4(a, lane);
}

// Work of wave w (of nw, the steering wave included) in the two triangular
// products: the T tile columns (W^T x) or tile rows (W x) ordered by size,
// T - s tiles for item s, are dealt in pairs {w, 2 nw - 1 - w} (an item past
// T is absent; T <= 2 nw - 2 for every m).  The sizes then total at most T
// per wave, and the waves sharing a SIMD (w and w + 4) carry nearly equal
// work.  Column item s is tile column s; row item s is tile row T - 1 - s.
__device__ __forceinline__ void mv_wt(const double* L, const double* x, int m, int T, int w, int nw, int lane,
                                      double& o1, double& o2) {
    w = __builtin_amdgcn_readfirstlane(w);  // the wave index is uniform: scalar tile loops
    const int s2 = 2 * nw - 1 - w;
    o1 = w < T ? wt_col(L, x, m, T, w, lane) : 0.0;
    o2 = s2 < T ? wt_col(L, x, m, T, s2, lane) : 0.0;
}
__device__ __forceinline__ void mv_wt_store(double* y, int m, int T, int w, int nw, int lane, double o1, double o2) {
    w = __builtin_amdgcn_readfirstlane(w);  // scalar offsets (nothing per lane to keep across the step loop)
    if ((lane & 3) == 0) {
        int l = lane >> 2;
        asm volatile("" : "+v"(l));
        const int s2 = 2 * nw - 1 - w;
        if (w < T && 16 * w + l < m) y[16 * w + l] = o1;
        if (s2 < T && 16 * s2 + l < m) y[16 * s2 + l] = o2;
    }
}
__device__ __forceinline__ void mv_w(const double* L, const double* x, int m, int T, int w, int nw, int lane,
                                     double& o1, double& o2) {
    w = __builtin_amdgcn_readfirstlane(w);
    const int i2 = T - 2 * nw + w;
    o1 = w < T ? w_strip(L, x, m, T - 1 - w, lane) : 0.0;
    o2 = i2 >= 0 ? w_strip(L, x, m, i2, lane) : 0.0;
}

// Entry of the Lanczos vectors that lane `lane` of wave w owns: the row of
// its W b output (w_strip leaves row 16 I + w_tiles_row(l) of tile row I in
// the four lanes l of a quad), lane & 3 == 0 for the wave's first tile row,
// lane & 3 == 1 for its second; -1 if none.  Every row below m has exactly
// one owner, which keeps q_j, q_{j-1} and the residual of that row.
__device__ __forceinline__ int owned_row(int m, int T, int w, int nw, int lane) {
    w = __builtin_amdgcn_readfirstlane(w);
    const int sel = lane & 3, rr = w_tiles_row(lane);
    const int I = sel == 0 ? T - 1 - w : T - 2 * nw + w;
    const bool has = sel == 0 ? w < T : (sel == 1 && I >= 0);
    const int r = 16 * I + rr;
    return has && r < m ? r : -1;
}

// Block sum with one barrier: the wave sums go to buf[0 .. nw - 1], which
// no thread reads or writes between the caller's previous barrier and this
// one, nor again before every thread has read the sum (a later barrier).
__device__ __forceinline__ double block_sum_once(double v, double* buf) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum_dpp(v);
    if (lane == 0) buf[wid] = v;
    lds_barrier();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += buf[i];
    return s;
}

// Scratch layout of the Lanczos phase (after the factor phase).
struct LzLayout {
    double *slot, *al, *be, *red, *sres;
};
__device__ __forceinline__ LzLayout lz_layout(double* scr, int kmax) {
    LzLayout o;
    o.slot = scr;                 // 2 MAXH (zero past m)
    o.al = scr + 2 * MAXH;        // kmax
    o.be = o.al + kmax;           // kmax + 1
    o.red = o.be + kmax + 1;      // 8
    o.sres = o.red + 8;           // 8: theta_min, r_min, theta_max, r_max, stop, k, total steps, rho
    return o;
}

// The pencil of one Lanczos run: C = W B W^T with W = L^{-1} in LDS and
// B = b0 B0 + b1 B1 (packed rows in HBM, B1 nullable).
struct LzCtx {
    int m, kmax, min_only, first_check;
    double tol;
    // a side whose Ritz value is below rho / loose_ratio in magnitude (rho the
    // spectral radius estimate) stops at the looser tol_loose: its value only
    // places the origin of a refining run (loose_ratio 0: off)
    double loose_ratio, tol_loose;
    const double* B0;
    double b0;
    const double* B1;
    double b1;
    double* Qg;        // this chain's basis (kmax x m)
    long long* prof;   // nullable: per-part cycles of the steering wave (slots 8..13), tests and passes (16, 17)
};

// Conditioning indicator of the factored pencil: the Cholesky pivots
// d_i = L_ii^2 lie in [lambda_min, lambda_max], so min d / max d (from the
// inverse's diagonal, W_ii = 1 / L_ii, in place after tri_inverse) is at
// least lambda_min / lambda_max; a value below the escalation threshold
// certainly means an ill-conditioned F.  Wave 0 reduces, `out` (LDS) passes
// the value to every thread (barrier included).
__device__ inline double pivot_ratio(const double* W, int m, double* out) {
    const int t = threadIdx.x, lane = t & 63;
    if (t < 64) {
        double lo = INFINITY, hi = 0.0;
        for (int i = lane; i < m; i += 64) {
            const double w = W[pk(i, i)];
            const double d = w * w;  // 1 / pivot
            lo = fmin(lo, d);
            hi = fmax(hi, d);
        }
        lo = wave_ext_dpp<false>(lo);
        hi = wave_ext_dpp<true>(hi);
        if (lane == 0) out[0] = lo / hi;  // min pivot / max pivot
    }
    lds_barrier();
    return out[0];
}

// A lower bound of the second smallest eigenvalue of T_k (al, be in LDS) for
// the Kato-Temple interval: multisection over [th, Gershgorin top] for the
// first point with two eigenvalues of T_k below it; returns the last point
// with fewer (the second Ritz value lies above it).  One wave, every lane
// with the same arguments; 4 passes of 64 points.
__device__ inline double second_ritz_lower(const double* al, const double* be, int k, double th, int lane) {
    double ghi = -INFINITY;
    for (int i = lane; i < k; i += 64) {
        const double rad = (i ? fabs(be[i]) : 0.0) + (i + 1 < k ? fabs(be[i + 1]) : 0.0);
        ghi = fmax(ghi, al[i] + rad);
    }
    ghi = wave_ext_dpp<true>(ghi);
    double lo = th, hi = ghi + 1e-14 * fabs(ghi) + 1e-300;
    if (!(hi > lo) || sturm_lds(al, be, k, lo) >= 2) return lo;
#pragma nounroll
    for (int it = 0; it < 4; ++it) {
        const double w = hi - lo;
        const double x = lo + w * ((double)(lane + 1) * (1.0 / 65.0));
        const unsigned long long mask = __ballot(sturm_lds(al, be, k, x) >= 2);
        const int first = mask ? __ffsll((long long)mask) - 1 : 64;
        const double nlo = lo + w * ((double)first * (1.0 / 65.0));
        const double nhi = first < 64 ? lo + w * ((double)(first + 1) * (1.0 / 65.0)) : hi;
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// Extreme eigenvalue(s) of C by Lanczos (lambda_min only when min_only),
// restarted from the Ritz vector after kmax steps, NCYCLES cycles at most.
// Every thread of the block calls it.  Results in sres (LDS): theta_min,
// r_min, theta_max, r_max, stop (1 converged, 2 not), steps of the last
// cycle, total steps, the spectral radius estimate of the last test; al / be
// hold T_k of the last cycle and Qg its basis.
// Wave 0 steers (Ritz values, residual bounds, stop decision); waves 1..
// hold B and run B a.  Every wave runs its share of the triangular products
// and owns the vector entries of its W b rows.  Both paths run the same
// sequence of barriers (eight per step).
__device__ __forceinline__ void lanczos_extreme(const double* L, double* scr, const LzCtx& c) {
    // the thread index is made opaque here so that lane addressing is formed
    // per call, not hoisted (and kept live) across a caller's loop
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    const int lane = t & 63, wv = t >> 6;
    const int m = c.m;
    const int tw = t - 64;
    const bool worker = wv >= 1;
    const int kmax = c.kmax;
    double* slot = scr;            // 2 MAXH (zero past m)
    double* al = scr + 2 * MAXH;   // kmax
    double* be = al + kmax;        // kmax + 1
    double* red = be + kmax + 1;   // 8
    double* sres = red + 8;        // 8: theta_min, r_min, theta_max, r_max, stop, k, total, rho
    double* Qg = c.Qg;
    for (int e = m + t; e < 2 * MAXH; e += blockDim.x) slot[e] = 0.0;
    // tile items of the triangular products (every wave, see mv_wt)
    const int T = (m + 15) >> 4, nwv = blockDim.x >> 6;
    // this lane's entry of the Lanczos vectors (see owned_row): q_j, q_{j-1}
    // and the residual of row orow stay in its registers, and alpha, beta and
    // the next vector are formed where W b leaves c
    const int orow = owned_row(m, T, wv, nwv, lane);
    const bool own = orow >= 0;
    // start vector (deterministic, positive)
    double qr = 0.0;
    if (own) {
        u4 hsh = philox10(u4{(uint32_t)orow, 0x5eedu, 0u, 0x51a7u}, 0x2010u, 0x3817u);
        qr = 0.5 + (double)(hsh.x >> 11) * (1.0 / 2097152.0);
    }
    double nq = block_sum_dpp(own ? qr * qr : 0.0, red);
    qr *= 1.0 / sqrt(nq);
    if (worker) {
        // B in registers: worker thread tw holds the block of rows 4 g .. 4 g + 3
        // (g = tw >> 3) and columns BC k8 .. BC k8 + BC - 1 (k8 = tw & 7), zero
        // past m, so that it reads only BC entries of a per product
        const int g = tw >> 3, k8 = tw & 7;
        double breg[MAXH];
#pragma unroll
        for (int i = 0; i < BR; ++i) {
#pragma unroll
            for (int k = 0; k < BC; ++k) {
                const int rr = BR * g + i, cc = BC * k8 + k;
                double v = 0.0;
                if (rr < m && cc < m) {
                    const int e = cc <= rr ? pk(rr, cc) : pk(cc, rr);
                    v = c.b0 * c.B0[e];
                    if (c.B1) v += c.b1 * c.B1[e];
                }
                breg[BC * i + k] = v;
            }
        }
        for (int cyc = 0;; ++cyc) {
        double qprev = 0.0, bprev = 0.0;
        for (int j = 0; j < kmax; ++j) {
            if (own) {
                Qg[(size_t)j * m + orow] = qr;
                slot[orow] = qr;
            }
            lds_barrier();  // B1
            // a = W^T q over this wave's tile columns
            double a1, a2;
            mv_wt(L, slot, m, T, wv, nwv, lane, a1, a2);
            lds_barrier();  // B2
            mv_wt_store(slot, m, T, wv, nwv, lane, a1, a2);
            lds_barrier();  // B3
            // b = B a from registers: four row sums over this thread's BC
            // columns, the loads of a one group of four ahead of the products
            // (the schedule pinned group by group so that the loads are not all
            // hoisted), then summed over the eight threads of the row block
            double bv;
            {
                double acc[BR] = {0.0, 0.0, 0.0, 0.0};
                const double* sv = slot + BC * k8;
                double cur[4], nxt[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) cur[u] = sv[u];
#pragma unroll
                for (int kk = 0; kk < BC; kk += 4) {
                    if (kk + 4 < BC) {
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (kk + 4 + u < BC) nxt[u] = sv[kk + 4 + u];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (kk + u < BC) {
#pragma unroll
                            for (int i = 0; i < BR; ++i) acc[i] += breg[BC * i + kk + u] * cur[u];
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < 4; ++u) cur[u] = nxt[u];
                }
                bv = red8x4(acc, lane);
            }
            lds_barrier();  // B4
            {
                // lanes 2 s and 2 s + 1 of the eight hold row 4 g + s
                const int rb = BR * g + ((lane >> 1) & 3);
                if ((lane & 1) == 0 && rb < m) slot[rb] = bv;
            }
            lds_barrier();  // B5
            // c = W b over this wave's tile rows; the owner lanes keep their row
            double cw1, cw2;
            mv_w(L, slot, m, T, wv, nwv, lane, cw1, cw2);
            double cv = (lane & 3) == 0 ? cw1 : cw2;
            // alpha = q^T c from the computed c, so that the new residual is
            // orthogonal to q to working precision whatever the conditioning of
            // W; the wave sums go to red (last read before the previous B7)
            const double alj = wave_uniform(block_sum_once(own ? qr * cv : 0.0, red));  // B6
            cv -= alj * qr + bprev * qprev;
            // beta: the wave sums go to the vector slot, which every wave has
            // finished reading (b) before B6
            const double bn = wave_uniform(sqrt(block_sum_once(own ? cv * cv : 0.0, slot)));  // B7
            lds_barrier();  // B8 (control wave stores alpha and beta and decides)
            if (sres[4] != 0.0) break;
            qprev = qr;
            qr = cv * (1.0 / bn);
            bprev = bn;
        }
        if (!(sres[4] == 2.0 && cyc + 1 < NCYCLES)) break;
        // not converged within kmax steps: restart from the Ritz vector(s)
        __syncthreads();  // basis rows in HBM are read across lanes
        {
            const int kk = (int)sres[5];
            double zr = own ? ritz_row(al, be, kk, sres[0], Qg, m, orow) : 0.0;
            if (!c.min_only && own) zr += ritz_row(al, be, kk, sres[2], Qg, m, orow);
            const double nz = block_sum_dpp(own ? zr * zr : 0.0, red);
            qr = zr * (1.0 / sqrt(nz));
        }
        lds_barrier();
        }
    } else {
        long long ph[6] = {0, 0, 0, 0, 0, 0};
        long long n_tests = 0, n_passes = 0, c_sect = 0, c_res = 0;
        if (lane == 0) sres[6] = 0.0;
        for (int cyc = 0;; ++cyc) {
        int next_check = c.first_check > 0 ? c.first_check : 4;
        double prev_q = -1.0;
        int prev_k = 0;
        double qprev = 0.0, bprev = 0.0;  // this wave's own rows (as the workers')
        // bracket of this lane's extreme Ritz value at the previous test (NaN: none)
        double w_lo = NAN, w_hi = NAN, w_r = 0.0;
        long long tprev = clock64();
#define PHASE(i)                          \
    {                                     \
const long long tn = clock64();   \
ph[i] += tn - tprev;              \
tprev = tn;                       \
    }
        for (int j = 0; j < kmax; ++j) {
            if (own) {
                Qg[(size_t)j * m + orow] = qr;
                slot[orow] = qr;
            }
            lds_barrier();  // B1
            PHASE(0)
            {
                double a1, a2;
                mv_wt(L, slot, m, T, 0, nwv, lane, a1, a2);
                lds_barrier();  // B2
                mv_wt_store(slot, m, T, 0, nwv, lane, a1, a2);
            }
            PHASE(1)
            lds_barrier();  // B3
            lds_barrier();  // B4
            PHASE(2)
            lds_barrier();  // B5
            double c1, c2;
            mv_w(L, slot, m, T, 0, nwv, lane, c1, c2);
            double cv = (lane & 3) == 0 ? c1 : c2;
            const double alj = wave_uniform(block_sum_once(own ? qr * cv : 0.0, red));  // B6
            PHASE(3)
            cv -= alj * qr + bprev * qprev;
            const double bn = wave_uniform(sqrt(block_sum_once(own ? cv * cv : 0.0, slot)));  // B7
            // T_k in LDS (this wave's own writes precede its reads below)
            if (lane == 0) {
                al[j] = alj;
                be[j + 1] = bn;
            }
            PHASE(4)
            const int k = j + 1;
            const bool exhausted = bn <= 1e-14 * fmax(fabs(al[0]), 1e-300);
            const bool check = exhausted || k == kmax || k >= next_check;
            double stop = 0.0;
            if (check) {
                ++n_tests;
                // T_k into registers
                const double aA = lane < k ? al[lane] : 0.0, aB = lane + 64 < k ? al[lane + 64] : 0.0;
                const double bA = lane < k ? be[lane] : 0.0, bB = lane + 64 < k ? be[lane + 64] : 0.0;
                const double bA1 = lane + 1 < k ? be[lane + 1] : 0.0, bB1 = lane + 65 < k ? be[lane + 65] : 0.0;
                const double b2A = bA * bA, b2B = bB * bB;
                const double rbA = bA != 0.0 ? 1.0 / bA : 0.0, rbB = bB != 0.0 ? 1.0 / bB : 0.0;
                // Gershgorin interval of T_k (rows spread over the lanes)
                double glo = INFINITY, ghi = -INFINITY;
                if (lane < k) {
                    const double rad = (lane ? fabs(bA) : 0.0) + fabs(bA1);
                    glo = aA - rad;
                    ghi = aA + rad;
                }
                if (lane + 64 < k) {
                    const double rad = fabs(bB) + fabs(bB1);
                    glo = fmin(glo, aB - rad);
                    ghi = fmax(ghi, aB + rad);
                }
                glo = wave_ext_dpp<false>(glo);
                ghi = wave_ext_dpp<true>(ghi);
                const double pad = 1e-14 * fmax(fabs(glo), fabs(ghi)) + 1e-300;
                glo -= pad;
                ghi += pad;
                // multisection: all lanes on lambda_min when only it is wanted, else
                // lanes 0-31 on lambda_min and 32-63 on lambda_max
                const int npts = c.min_only ? 64 : 32;
                const bool want_min = c.min_only || lane < 32;
                const int sub = c.min_only ? lane : (lane & 31);
                double lo = glo, hi = ghi;
                // warm start: T_k's leading submatrices are the earlier T's, so by
                // interlacing theta_min can only fall and theta_max only rise since
                // the last test.  Keep the previous inner end; take the outer end a
                // little beyond the previous bracket if a Sturm count confirms no
                // eigenvalue lies past it.
                if (w_lo == w_lo) {
                    const double span = 4.0 * w_r + 16.0 * (w_hi - w_lo) + 1e-12 * fmax(fabs(w_lo), fabs(w_hi));
                    const double xw = want_min ? w_lo - span : w_hi + span;
                    const int cw = sturm_lds(al, be, k, xw);
                    ++n_passes;
                    const bool okw = want_min ? (cw == 0) : (cw >= k);
                    if (okw) {
                        if (want_min) {
                            lo = fmax(glo, xw);
                            hi = fmin(ghi, w_hi);
                        } else {
                            lo = fmax(glo, w_lo);
                            hi = fmin(ghi, xw);
                        }
                        if (!(hi > lo)) {
                            lo = glo;
                            hi = ghi;
                        }
                    }
                }
                // multisection down to a relative width rel (at most 12 passes);
                // the points lo + w (i / (npts + 1)) and the new ends use the one
                // expression, so each new end is exactly a point that was counted
                const double inv = 1.0 / (double)(npts + 1);
                auto msect = [&](double rel) {
#pragma nounroll
                    for (int it = 0; it < 12; ++it) {
                        const double w = hi - lo;
                        if (!(w > rel * fmax(fabs(lo), fabs(hi)))) break;
                        const double x = lo + w * ((double)(sub + 1) * inv);
                        const int cnt = sturm_lds(al, be, k, x);
                        ++n_passes;
                        const bool hitp = want_min ? (cnt >= 1) : (cnt >= k);
                        const unsigned long long mask = __ballot(hitp);
                        unsigned long long hm;
                        if (c.min_only) hm = mask;
                        else hm = want_min ? (mask & 0xffffffffull) : (mask >> 32);
                        const int first = hm ? __ffsll((long long)hm) - 1 : npts;
                        const double nlo = lo + w * ((double)first * inv);
                        const double nhi = first < npts ? lo + w * ((double)(first + 1) * inv) : hi;
                        lo = nlo;
                        hi = nhi;
                    }
                };
                const int src_max = c.min_only ? 0 : 32;
                double th = 0.0, res = 0.0, thmin = 0.0, thmax = 0.0, tmin = 0.0, tmax = 0.0;
                bool conv_now = false;
                // residual bound below tol |theta|, or at the rounding level of C
                // (scaled by the spectral radius: Gershgorin bound of T_k, which
                // also covers lambda_max when only lambda_min is tracked).  The
                // bound hardly depends on theta once theta is far closer to the
                // Ritz value than the gap, so the test runs with theta to 1e-10
                // (relative) and a passing test (or the last step) is repeated
                // with theta to the rounding level.
                double rmin = 0.0, rmax = 0.0, rho_last = 0.0;
                auto test = [&]() {
                    th = 0.5 * (lo + hi);
                    res = exhausted ? 0.0 : fabs(bn) * backward_norm_lds(al, be, k, th);
                    thmin = __shfl(th, 0, 64);
                    thmax = __shfl(th, src_max, 64);
                    rmin = __shfl(res, 0, 64);
                    rmax = __shfl(res, src_max, 64);
                    const double rho = fmax(fmax(fabs(thmin), c.min_only ? 0.0 : fabs(thmax)),
                                            fmax(fabs(glo), fabs(ghi)));
                    const double floor_r = 2.2e-14 * rho;
                    tmin = fmax(c.tol * fabs(thmin), floor_r);
                    tmax = fmax(c.tol * fabs(thmax), floor_r);
                    if (c.loose_ratio > 0.0) {
                        if (rho > c.loose_ratio * fabs(thmin)) tmin = fmax(tmin, c.tol_loose * fabs(thmin));
                        if (!c.min_only && rho > c.loose_ratio * fabs(thmax))
                            tmax = fmax(tmax, c.tol_loose * fabs(thmax));
                    }
                    rho_last = rho;
                    const bool cmin = rmin <= tmin;
                    const bool cmax = c.min_only || rmax <= tmax;
                    conv_now = exhausted || (cmin && cmax);
                };
                long long tq = clock64();
                msect(1e-10);
                long long tr = clock64();
                c_sect += tr - tq;
                test();
                tq = clock64();
                c_res += tq - tr;
                if (conv_now || k == kmax) {
                    msect(2e-16);
                    tr = clock64();
                    c_sect += tr - tq;
                    test();
                    c_res += clock64() - tr;
                }
                w_lo = lo;
                w_hi = hi;
                w_r = res;
                if (lane == 0) {
                    sres[0] = th;
                    sres[1] = res;
                    sres[7] = rho_last;
                }
                if (lane == src_max) {
                    sres[2] = c.min_only ? NAN : th;
                    sres[3] = c.min_only ? 0.0 : res;
                }
                if (conv_now) stop = 1.0;
                else if (k == kmax) stop = 2.0;
                // next test: where the residual decay since the last test predicts
                // convergence (at least 2, at most 12 steps ahead)
                double q = rmin / tmin;
                if (!c.min_only) q = fmax(q, rmax / tmax);
                int ahead = 4;
                if (prev_q > 0.0 && q < prev_q && q > 1.0) {
                    const double rate = log(q / prev_q) / (double)(k - prev_k);  // < 0
                    ahead = (int)ceil(log(q) / -rate);
                }
                ahead = ahead < 2 ? 2 : (ahead > 12 ? 12 : ahead);
                prev_q = q;
                prev_k = k;
                next_check = k + ahead;
            } else if (k == kmax) {
                stop = 2.0;
            }
            if (lane == 0) {
                sres[4] = stop;
                sres[5] = (double)k;
                if (stop != 0.0) sres[6] += (double)k;
            }
            lds_barrier();  // B8
            PHASE(5)
            if (stop != 0.0) break;
            qprev = qr;
            qr = cv * (1.0 / bn);
            bprev = bn;
        }
        if (!(sres[4] == 2.0 && cyc + 1 < NCYCLES)) break;
        __syncthreads();  // basis rows in HBM are read across lanes
        {
            const int kk = (int)sres[5];
            double zr = own ? ritz_row(al, be, kk, sres[0], Qg, m, orow) : 0.0;
            if (!c.min_only && own) zr += ritz_row(al, be, kk, sres[2], Qg, m, orow);
            const double nz = block_sum_dpp(own ? zr * zr : 0.0, red);
            qr = zr * (1.0 / sqrt(nz));
        }
        lds_barrier();
        }
#undef PHASE
        if (c.prof && t == 0) {
            for (int i = 0; i < 6; ++i) c.prof[8 + i] = ph[i];
            c.prof[16] = n_tests;
            c.prof[17] = n_passes;
            c.prof[18] = c_sect;
            c.prof[19] = c_res;
        }
    }
}

// Kernel vector of the pencil at its root: u = W^T z with z the Ritz vector
// of lam from the last Lanczos run (k steps, basis Qg), written to u (m) and
// the packed vec(u u^T) (off-diagonal entries doubled) to U2, the left
// operand of the normal GEMM w_i = u^T A_i u.  Every thread calls it.
__device__ __forceinline__ void ritz_u(const double* L, double* scr, int m, int kmax, int k, double lam,
                                       const double* Qg, double* u, double* U2) {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));  // per-call lane addressing (see lanczos_extreme)
    const int wv = t >> 6;
    const int tw = t - 64;
    const int r = tw >> 1, h = tw & 1;
    const bool own = wv >= 1 && r < m;
    const int R0w = 32 * (wv - 1);
    const LzLayout lz = lz_layout(scr, kmax);
    double* slot = lz.slot;
    const double zr = own ? ritz_row(lz.al, lz.be, k, lam, Qg, m, r) : 0.0;
    lds_barrier();
    if (own && h == 0) slot[r] = zr;
    lds_barrier();
    double uv = own ? wt_column(L, slot, r, R0w, m, h) : 0.0;
    uv += __shfl_xor(uv, 1, 64);
    lds_barrier();
    if (own && h == 0) {
        u[r] = uv;
        slot[r] = uv;
    }
    lds_barrier();
    // packed u u^T with the off-diagonal entries doubled, consecutive packed
    // indices on consecutive threads (coalesced stores)
    if (wv >= 1) {
        const int nt = blockDim.x - 64, P = m * (m + 1) / 2;
        for (int e = tw; e < P; e += nt) {
            int rr = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
            while (rr * (rr + 1) / 2 > e) --rr;
            while ((rr + 1) * (rr + 2) / 2 <= e) ++rr;
            const int cc = e - rr * (rr + 1) / 2;
            U2[e] = (cc == rr ? 1.0 : 2.0) * slot[rr] * slot[cc];
        }
    }
}

// One chain's line oracle (the body of k_line_fused); every thread of the
// block calls it with the same arguments.
//
// Far-root refinement.  The rounding error of C = L^-1 B L^-T is about eps
// times its spectral radius rho, so the root whose eigenvalue is small
// against rho (the far root of a start next to the boundary, rho ~ 1/|t-|)
// comes out of the run from x with a relative error near eps rho / |lambda|.
// When a run from the plain origin ends with rho > refine_ratio |lambda| for
// a root that decides the result, that side's Lanczos test uses the loose
// tolerance, the chain is queued (rlist) with the new origin
// t0 = t1 (1 - 2^-10) (t1 the root found; negative for t-), and a second,
// REFINE, pass factors F(x + t0 v) (which certifies t0 inside) and runs
// Lanczos on the shifted pencil, where that root's eigenvalue
// -1/(t1 - t0) dominates the spectrum (lambda_min only; lambda_max as
// -lambda_min of -C).  If the factor at t0 does not exist, the origin backs
// off (see below) before the REFINE pass repeats the plain solve from x at
// the full tolerance (REFINE_FAILED).
template <bool REFINE>
__device__ __forceinline__ void line_fused_chain(const FusedArgs& a, int chain, double* lds) {
    const int m = a.m, P = a.P, md = a.md;
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
    // F(x) carried over from the walk's previous round: formed from (Fp, Bp,
    // us) wherever F is read, and written to this chain's F row
    const bool upd = !REFINE && a.upd_F != nullptr;
    double us = 0.0;
    const double *Fp = nullptr, *Bp = nullptr;
    double* Fo = nullptr;
    if (upd) {
        us = a.upd_s[chain];
        if (!(us == us)) {  // moved off its line: no F(x) until the next full assembly
            if (t == 0) {
                a.status[chain] = WALK_STALE;
                a.tm[chain] = NAN;
                a.tp[chain] = NAN;
                a.hit[chain] = HIT_NONE;
                if (a.flags) a.flags[chain] = 0;
                if (a.lam) {
                    for (int i = 0; i < 4; ++i) a.lam[4 * chain + i] = 0.0;
                }
            }
            return;
        }
        Fp = a.upd_F + (size_t)chain * a.ldfb;
        Bp = a.upd_B + (size_t)chain * a.ldfb;
        Fo = const_cast<double*>(Fr);
    }
    double t0 = a.shift ? a.shift[chain] : 0.0;
    if (REFINE) {
        if (!isfinite(t0)) t0 = 0.0;
    } else if (!(t0 > 0.0) || !isfinite(t0)) {
        t0 = 0.0;  // no usable bracket: plain origin
    }
    const int side = t0 < 0.0 ? 2 : 1;  // REFINE: the root refined from t0
    int flags = 0;
    // Kato-Temple interval of the dense t+ (wave 0, lane 0 keeps it)
    bool kt_set = false;
    double kt_lo = NAN;
    int32_t st = SPEC_OK;
    long long* prof = a.prof ? a.prof + (size_t)chain * SPEC_DIAG_PHASE_SLOTS : nullptr;
#define STAMP(i) \
    if (prof && t == 0) prof[i] = clock64();
    STAMP(0)

    // ---- diagonal rows: ratio test from x (ties of the smallest root flagged:
    // bit 1 of `bad`, which carries the not-interior test in bit 0)
    double dtp = INFINITY, dtm = -INFINITY;
    int dj = -1, bad = 0;
    for (int j = t; j < md; j += blockDim.x) {
        double f;
        if (upd) {
            f = fma(us, Bp[P + j], Fp[P + j]);
            Fo[P + j] = f;
        } else {
            f = Fr[P + j];
        }
        const double b = a.membership_only ? 0.0 : Br[P + j];
        if (!(f > 0.0)) bad |= 1;
        const double r = b / f;
        if (r < 0.0) {
            const double tt = -1.0 / r;
            if (tt < dtp) {
                dtp = tt;
                dj = j;
                bad &= 1;
            } else if (tt == dtp) {
                bad |= 2;
            }
        } else if (r > 0.0) {
            dtm = fmax(dtm, -1.0 / r);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double otp = __shfl_xor(dtp, o, 64);
        const int oj = __shfl_xor(dj, o, 64);
        const int ob = __shfl_xor(bad, o, 64);
        const int nb = (bad | ob) & 1;
        if (otp < dtp) {
            dtp = otp;
            dj = oj;
            bad = nb | (ob & 2);
        } else if (otp == dtp && oj >= 0 && dj >= 0) {
            if (oj < dj) dj = oj;
            bad = nb | 2;
        } else {
            bad = nb | (bad & 2);
        }
        dtm = fmax(dtm, __shfl_xor(dtm, o, 64));
    }
    if (lane == 0) { rtp[wv] = dtp; rtm[wv] = dtm; rj[wv] = dj; rbad[wv] = bad; }
    lds_barrier();
    dtp = INFINITY; dtm = -INFINITY; dj = -1; bad = 0;
    for (int w = 0; w < nw; ++w) {
        const int wb = rbad[w];
        if (rtp[w] < dtp) {
            dtp = rtp[w];
            dj = rj[w];
            bad = (bad & 1) | wb;
        } else if (rtp[w] == dtp && rj[w] >= 0 && dj >= 0) {
            if (rj[w] < dj) dj = rj[w];
            bad = (bad | wb) | 2;
        } else {
            bad |= wb & 1;
        }
        dtm = fmax(dtm, rtm[w]);
    }
    lds_barrier();
    const bool dtie = (bad & 2) != 0;
    bad &= 1;
    // reduced-precision pencils that are not definite at the plain origin are
    // decided by the FP64 pass (their rounding can move a start next to the
    // boundary outside)
    if (!REFINE && bad && a.elist) {
        if (t == 0) a.elist[atomicAdd(a.ecount, 1)] = chain;
        return;
    }
    double tp = dtp, tm = dtm;
    int hit = dj >= 0 ? dj : HIT_NONE;
    double lmin = 0.0, lmax = 0.0;
    int iters = 0;
    bool conv = true;
    int cert = 0;

    if (bad) st = SPEC_NOT_INTERIOR;
    if (!bad && m > 0) {
        // ---- factor F0 = F + t0 B.  A factor at t0 > 0 certifies t0 < t+; when
        // it does not exist the bracket is discarded and F(x) is factored.  With
        // an upper end t_hi, F(x + t_hi v) is tested first (a definite F there
        // means the bracket missed t+ on the high side: counted, harmless).
        // One loop so that the factorisation is instantiated once.
        // REFINE: t0 = t1 (1 - 2^-10); should the factor not exist there (t1 too
        // far out: the first pass stopped at the loose tolerance), the origin
        // backs off to t1 (1 - 2^-5), then t1 / 2, before the plain solve
        int phase = a.shift_hi ? 0 : 1;
        bool ok = false;
        int tries = 0;
        const double t1r = t0 / (1.0 - 0.0009765625);
        long long cst[4] = {0, 0, 0, 0};  // Cholesky stage cycles (profiling)
        STAMP(1)
        for (;;) {
            const double sh = phase == 0 ? a.shift_hi[chain] : t0;
            const double* Bs = a.membership_only || sh == 0.0 ? nullptr : Br;
            if (upd) fill_pencil_upd(L, Fp, Bp, us, Fo, Bs, sh, P, t, blockDim.x);
            else fill_pencil(L, Fr, Bs, sh, P, t, blockDim.x);
            lds_barrier();
            ok = chol_blocked(L, m, scr, sflag, prof ? cst : nullptr);
            lds_barrier();
            if (phase == 0) {
                if (ok) cert = 2;
                phase = 1;
                continue;
            }
            if (ok || t0 == 0.0) break;
            if (REFINE) {
                if (tries < 2) {
                    ++tries;
                    t0 = t1r * (tries == 1 ? 1.0 - 0.03125 : 0.5);
                    continue;
                }
                flags |= SPEC_FLAG_REFINE_FAILED;
            } else {
                cert = 1;
            }
            t0 = 0.0;
        }
        STAMP(2)
        if (prof && t == 0) {
            prof[7] = cst[0];
            prof[14] = cst[1];
            prof[15] = cst[2];
            prof[23] = cst[3];
        }
        if (prof && t == 64) prof[20] = cst[3];
        long long ist[3] = {0, 0, 0};  // triangular-inverse part cycles (profiling)
        if (!REFINE && !ok && a.elist) {
            if (t == 0) a.elist[atomicAdd(a.ecount, 1)] = chain;
            return;
        }
        if (ok && !a.membership_only) tri_inverse(L, m, scr, prof ? ist : nullptr);
        // reduced-precision pencils of an ill-conditioned F are passed on to an
        // FP64 assembly (the chain is queued; that pass writes its results)
        if (!REFINE && ok && !a.membership_only && a.elist && t0 == 0.0) {
            const double pr = pivot_ratio(L, m, rtp);
            if (pr < a.esc_ratio) {
                if (t == 0) a.elist[atomicAdd(a.ecount, 1)] = chain;
                return;
            }
        }
        if (prof && t == 0) {
            prof[21] = ist[1];
            prof[22] = ist[2];
        }
        STAMP(3)
        if (!ok) st = SPEC_NOT_INTERIOR;
        if (ok && !a.membership_only) {
            const int hm = (m + 1) >> 1;
            const int tw = t - 64;
            const int r = tw >> 1, h = tw & 1;
            const bool own = wv >= 1 && r < m;
            (void)hm;
            const int kmax = a.kmax;
            const LzLayout lz = lz_layout(scr, kmax);
            double* slot = lz.slot;
            double* al = lz.al;
            double* be = lz.be;
            double* sres = lz.sres;
            double* Qg = a.Q + (size_t)chain * a.ldq;
            STAMP(4)
            // REFINE from a shifted origin: one side (lambda_max(C) = -lambda_min(-C))
            const bool shifted = REFINE && t0 != 0.0;
            LzCtx lc;
            lc.m = m;
            lc.kmax = kmax;
            lc.min_only = shifted ? 1 : a.min_only;
            lc.first_check = a.first_check;
            lc.tol = a.tol;
            lc.loose_ratio = (!REFINE && t0 == 0.0) ? a.refine_ratio : 0.0;
            lc.tol_loose = a.tol_loose;
            lc.B0 = Br;
            lc.b0 = (shifted && side == 2) ? -1.0 : 1.0;
            lc.B1 = nullptr;
            lc.b1 = 0.0;
            lc.Qg = Qg;
            lc.prof = prof;
            lanczos_extreme(L, scr, lc);
            __syncthreads();  // basis entries in HBM are read across lanes below
            STAMP(5)
            lmin = sres[0];
            lmax = sres[2];
            conv = sres[4] == 1.0;
            const int k = (int)sres[5];
            iters = (int)sres[6];
            if (REFINE && a.lam) iters += (int)a.lam[4 * chain + 3];  // steps of the first pass
            // dense block: roots measured from the origin t0
            double dtpd = INFINITY, dtmd = -INFINITY;
            if (!shifted) {
                if (lmax > 0.0) dtmd = t0 - 1.0 / lmax;
                if (lmin < 0.0) dtpd = t0 - 1.0 / lmin;
                if (a.min_only) dtmd = NAN;  // lambda_max is not converged by design
            }
            int rside = 0;  // first pass: the root to refine (1 t+, 2 t-)
            if (!REFINE && t0 == 0.0 && a.refine_ratio > 0.0 && conv && a.rlist) {
                const double rho = sres[7];
                if (lmin < 0.0 && rho > a.refine_ratio * fabs(lmin) && dtpd <= dtp * (1.0 + 1e-6))
                    rside = 1;
                else if (!a.min_only && !a.want_vec && lmax > 0.0 && rho > a.refine_ratio * lmax &&
                         dtmd >= dtm * (1.0 + 1e-6))
                    rside = 2;
                if (rside && t == 0) {
                    const double t1 = rside == 1 ? dtpd : dtmd;
                    a.rshift[chain] = t1 * (1.0 - 0.0009765625);
                    const int slot = atomicAdd(a.rcount, 1);
                    a.rlist[slot] = make_int2(a.inst_id, chain);
                }
            }
            if (shifted) {
                // the refined root from t0; the other one stays that of the first pass
                if (side == 1) {
                    if (lmin < 0.0) dtpd = t0 - 1.0 / lmin;
                    tm = a.tm[chain];
                    if (dtpd <= tp) {
                        tp = dtpd;
                        hit = HIT_DENSE;
                    }
                } else {
                    if (lmin < 0.0) dtmd = t0 + 1.0 / lmin;  // lambda_max(C) = -lmin
                    lmax = -lmin;
                    tm = fmax(tm, dtmd);
                    tp = a.tp[chain];
                    hit = a.hit[chain];
                }
            } else {
                tm = isnan(dtmd) ? dtmd : fmax(tm, dtmd);
                if (dtpd <= tp) {
                    tp = dtpd;
                    hit = HIT_DENSE;
                }
            }
            // a posteriori interval of the dense t+ from the run that fixes it
            // (Kato-Temple): lambda_min lies in [theta - d, theta] with
            // d = r^2 / (theta_2 - theta), r the residual bound plus the
            // rounding level 8 eps rho, theta_2 bounded below by multisection on
            // T_k; t+ = t0 - 1/lambda then lies in [t0 - 1/(theta - d), t0 - 1/theta]
            const bool fixes_tp = rside != 1 && !(shifted && side == 2);
            if (fixes_tp) {
                kt_set = true;
                if (wv == 0 && lmin < 0.0 && conv && k >= 3) {
                    const double th2 = second_ritz_lower(lz.al, lz.be, k, lmin, lane);
                    const double r = sres[1] + 8.0 * 2.220446049250313e-16 * sres[7];
                    const double gap = th2 - lmin;
                    if (gap > 0.0 && isfinite(r)) {
                        const double d = r * r / gap;
                        kt_lo = t0 - 1.0 / (lmin - d);
                    }
                }
            }
            // the kernel vector of a t+ hit comes from the run that fixes t+
            const bool need_vec = a.want_vec && fixes_tp && hit == HIT_DENSE && isfinite(tp) &&
                                  (a.ell == nullptr || tp < a.ell[chain]);
            // a reflection from reduced-precision pencils: the hit point (pulled
            // back by a relative 1e-6) and the normal need the FP64 root
            if (!REFINE && need_vec && a.elist) {
                if (t == 0) a.elist[atomicAdd(a.ecount, 1)] = chain;
                return;
            }
            if (need_vec)
                ritz_u(L, scr, m, kmax, k, lmin, Qg, a.u + (size_t)chain * a.ldu, a.U2 + (size_t)chain * a.ldu2);
            if (rside) flags |= SPEC_FLAG_REFINED;
        }
    }
    STAMP(6)
#undef STAMP
    if (t == 0) {
        if (st == SPEC_NOT_INTERIOR) {
            tm = NAN;
            tp = NAN;
            hit = HIT_NONE;
        } else if (st == SPEC_OK && !a.membership_only) {
            if (!conv) st = SPEC_NOCONV;
            else if (isinf(tp) || isinf(tm)) st = SPEC_UNBOUNDED;
        }
        // t+ attained by two pieces of the boundary: two diagonal rows, or a
        // diagonal row and the dense block (exact ties, as the oracle's)
        if (isfinite(tp) && ((hit >= 0 && dtie) || (hit == HIT_DENSE && tp == dtp))) flags |= SPEC_FLAG_TIE;
        // certified interval of t+: a diagonal row's ratio is exact; a dense
        // hit carries the Kato-Temple interval, certified when it is within
        // 2e-9 t+ (an uncertified value is still the Lanczos value)
        if ((kt_set || (!REFINE && hit != HIT_DENSE)) && st != SPEC_NOT_INTERIOR && !a.membership_only) {
            double lo = tp, hi = tp;
            if (hit == HIT_DENSE) {
                // the returned value is the upper end; no certified lower end
                // (-inf) when T_k gave no gap or the run did not converge
                lo = kt_lo == kt_lo ? kt_lo : -INFINITY;
                hi = tp;
                if (!(hi - lo <= 2e-9 * fabs(hi))) flags |= SPEC_FLAG_UNCERTIFIED;
            }
            if (a.cert) {
                a.cert[2 * chain] = lo;
                a.cert[2 * chain + 1] = hi;
            }
        } else if (!REFINE && a.cert) {
            // none (no dense root computed, or one the refining pass fixes)
            a.cert[2 * chain] = NAN;
            a.cert[2 * chain + 1] = NAN;
        }
        const int keep = kt_set ? ~(SPEC_FLAG_REFINE_FAILED | SPEC_FLAG_TIE | SPEC_FLAG_UNCERTIFIED)
                                : ~(SPEC_FLAG_REFINE_FAILED | SPEC_FLAG_TIE);
        if (REFINE && a.flags) flags |= a.flags[chain] & keep;
        if (REFINE && (flags & SPEC_FLAG_CERT_FALLBACK)) cert = 1;  // from the first pass
        if (st == SPEC_OK && cert) st = SPEC_CERT_FALLBACK;  // informational: values are final
        if (a.escalated) flags |= SPEC_FLAG_ESCALATED;
        if (a.flags) a.flags[chain] = flags | (cert == 1 ? SPEC_FLAG_CERT_FALLBACK : 0);
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

__global__ __launch_bounds__(512) void k_line_fused(FusedArgs a) {
    extern __shared__ double lds[];
    const int chain = a.idx ? a.idx[blockIdx.x] : (int)blockIdx.x;
    line_fused_chain<false>(a, chain, lds);
}

// The REFINE pass over the chains the first pass queued: persistent
// workgroups take items (instance, chain) of `work` from an atomic counter
// until *nwork (written by the first pass) is reached.  MULTI: args holds one
// FusedArgs per instance (the REFINE pass's: shift = the queued origins);
// otherwise `one` serves every item.
template <bool MULTI>
__global__ __launch_bounds__(512) void k_line_refine(FusedArgs one, const FusedArgs* __restrict__ args,
                                                     const int2* __restrict__ work, const int* __restrict__ nwork,
                                                     int* __restrict__ counter) {
    extern __shared__ double lds[];
    const int total = *nwork;
    for (;;) {
        // the item goes through the first LDS word, between chains (no static
        // LDS: a chain of the largest size uses all of it)
        __syncthreads();  // the previous item is finished with LDS
        if (threadIdx.x == 0) ((int*)lds)[0] = atomicAdd(counter, 1);
        __syncthreads();
        const int it = ((int*)lds)[0];
        __syncthreads();  // every thread has read it before the chain writes LDS
        if (it >= total) break;
        const int2 w = work[it];
        if (MULTI) line_fused_chain<true>(args[w.x], w.y, lds);
        else line_fused_chain<true>(one, w.y, lds);
    }
}

// Persistent form over many spectrahedra: workgroups take (instance, chain)
// items from `work` in order (an atomic counter hands them out, so the
// longest items, placed first, start first) until the list is exhausted.
// The dynamic LDS is sized for the largest instance.
__global__ __launch_bounds__(512) void k_line_fused_multi(const FusedArgs* __restrict__ args,
                                                          const int2* __restrict__ work, int nwork,
                                                          int* __restrict__ counter) {
    extern __shared__ double lds[];
    for (;;) {
        // the item goes through the first LDS word, between chains (no static
        // LDS: a chain of the largest size uses all of it)
        __syncthreads();  // the previous item is finished with LDS
        if (threadIdx.x == 0) ((int*)lds)[0] = atomicAdd(counter, 1);
        __syncthreads();
        const int it = ((int*)lds)[0];
        __syncthreads();  // every thread has read it before the chain writes LDS
        if (it >= nwork) break;
        const int2 w = work[it];
        line_fused_chain<false>(args[w.x], w.y, lds);
    }
}

// Two-sided Cholesky certificate of a dense t+ (one workgroup per chain, the
// thread and LDS shape of k_line_fused): F(x + t v) = F + t B must have a
// factor at t = t+ (1 - 1e-9) and none at t+ (1 + 1e-9), which places the
// boundary within 1e-9 t+ of the returned value up to the factorisations'
// own rounding.  A failure sets SPEC_FLAG_CHOL_CERT_FAILED; values and
// statuses are left as they are.
__global__ __launch_bounds__(512) void k_line_certify(FusedArgs a) {
    extern __shared__ double lds[];
    const int chain = blockIdx.x;
    const int m = a.m, P = a.P;
    const int32_t st = a.status[chain];
    const double tp = a.tp[chain];
    if (!(st == SPEC_OK || st == SPEC_NONSMOOTH || st == SPEC_CERT_FALLBACK) || a.hit[chain] != HIT_DENSE ||
        !isfinite(tp) || m == 0)
        return;
    double* L = lds;
    double* scr = lds + P;
    int* sflag = (int*)(scr + 256);
    const double* Fr = a.FB + (size_t)chain * a.ldfb;
    const double* Br = a.FB + (size_t)(a.brow0 + chain) * a.ldfb;
    bool pass = true;
    for (int s = 0; s < 2; ++s) {
        const double tc = tp * (s == 0 ? 1.0 - 1e-9 : 1.0 + 1e-9);
        fill_pencil(L, Fr, Br, tc, P, threadIdx.x, blockDim.x);
        lds_barrier();
        const bool ok = __builtin_amdgcn_readfirstlane((int)chol_blocked(L, m, scr, sflag)) != 0;
        lds_barrier();
        pass = pass && (s == 0 ? ok : !ok);
    }
    if (threadIdx.x == 0 && a.flags) {
        if (pass) a.flags[chain] &= ~SPEC_FLAG_CHOL_CERT_FAILED;
        else a.flags[chain] |= SPEC_FLAG_CHOL_CERT_FAILED;
    }
}

__global__ void k_zero_int(int* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__global__ void k_zero_ints(int* p, int count) {
    if (blockIdx.x == 0 && (int)threadIdx.x < count) p[threadIdx.x] = 0;
}

int line_fused_multi_blocks_per_cu(int max_m, int kmax) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_line_fused_multi),
                                                     fused_threads(max_m), fused_lds_bytes(max_m, kmax)) !=
        hipSuccess)
        per_cu = 1;
    return per_cu;
}

hipError_t launch_line_fused_multi(const FusedArgs* args, const int2* work, int nwork, int* counter, int max_m,
                                   int kmax, int nblocks, hipStream_t s) {
    if (nwork <= 0) return hipSuccess;
    if (max_m > 2 * MAXH) return hipErrorInvalidValue;
    const size_t lds = fused_lds_bytes(max_m, kmax);
    if (lds > 163840) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, counter);
    hipLaunchKernelGGL(k_line_fused_multi, dim3(nblocks), dim3(fused_threads(max_m)), lds, s, args, work, nwork,
                       counter);
    return hipGetLastError();
}

// Smallest s > 0 with 1 + a s + b s^2 = 0 (+inf when there is none): the
// root 2 / (-a + sqrt(a^2 - 4 b)) in the form without cancellation.
__device__ __forceinline__ double first_root_q(double a, double b) {
    if (b > 0.0 && !(a < 0.0)) return INFINITY;
    const double disc = a * a - 4.0 * b;
    if (disc < 0.0) return INFINITY;
    const double den = -a + sqrt(disc);
    return den > 0.0 ? 2.0 / den : INFINITY;
}

// One workgroup per chain, the thread and LDS shape of k_line_fused.  For the
// dense block, certified Weyl stepping (the degree-2 case of Lemma "PEP and S
// cap C"): at tau_k, L L^T = Q(tau_k), D1 = L^-1 (Q1 + 2 tau_k Q2) L^-T and
// D2 = L^-1 Q2 L^-T; by Weyl's inequality lambda_min(Q(tau_k + s)) >= 0 while
// 1 + d1 s + d2 s^2 > 0 with d1, d2 lower bounds of lambda_min(D1),
// lambda_min(D2) (Ritz value minus residual bound), so tau_{k+1} = tau_k + s*
// with s* that polynomial's first positive root.  Stop when the step falls
// below 1e-15 tau, when the factor no longer exists (rounding level), or past
// the horizon.  Diagonal rows: scalar quadratics.
__global__ __launch_bounds__(512) void k_curve2(CurveArgs a) {
    extern __shared__ double lds[];
    const int m = a.m, P = a.P, md = a.md;
    const int row = blockIdx.x;                      // pencil rows of this workgroup
    const int chain = a.idx ? a.idx[row] : row;     // its chain (outputs, basis, horizon)
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
    double* L = lds;
    double* scr = lds + P;
    int* sflag = (int*)(scr + 256);
    double* rtp = scr + 264;
    double* rtm = rtp + 8;
    int* rj = (int*)(rtm + 8);
    int* rbad = rj + 8;
    const double* Q0 = a.FB + (size_t)row * a.ldfb;
    const double* Q1 = a.FB + (size_t)(a.brow0 + row) * a.ldfb;
    const double* Q2 = a.FB + (size_t)(2 * a.brow0 + row) * a.ldfb;
    const double hz = a.horizon ? a.horizon[chain] : a.hscalar;
    int32_t st = SPEC_OK;

    // ---- diagonal rows: first roots of q0 + q1 t + q2 t^2 on both sides
    double dtp = INFINITY, dtm = INFINITY;  // dtm: distance on the negative side
    int dj = -1, bad = 0;
    for (int j = t; j < md; j += blockDim.x) {
        const double q0 = Q0[P + j], q1 = Q1[P + j], q2 = Q2[P + j];
        if (!(q0 > 0.0)) bad = 1;
        const double sp = first_root_q(q1 / q0, q2 / q0);
        if (sp <= hz && sp < dtp) { dtp = sp; dj = j; }
        if (a.both) {
            const double sm = first_root_q(-q1 / q0, q2 / q0);
            if (sm <= hz) dtm = fmin(dtm, sm);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double otp = __shfl_xor(dtp, o, 64);
        const int oj = __shfl_xor(dj, o, 64);
        if (otp < dtp || (otp == dtp && oj >= 0 && (dj < 0 || oj < dj))) { dtp = otp; dj = oj; }
        dtm = fmin(dtm, __shfl_xor(dtm, o, 64));
        bad |= __shfl_xor(bad, o, 64);
    }
    if (lane == 0) { rtp[wv] = dtp; rtm[wv] = dtm; rj[wv] = dj; rbad[wv] = bad; }
    lds_barrier();
    dtp = INFINITY; dtm = INFINITY; dj = -1; bad = 0;
    for (int w = 0; w < nw; ++w) {
        if (rtp[w] < dtp || (rtp[w] == dtp && rj[w] >= 0 && (dj < 0 || rj[w] < dj))) { dtp = rtp[w]; dj = rj[w]; }
        dtm = fmin(dtm, rtm[w]);
        bad |= rbad[w];
    }
    lds_barrier();
    double tp = dtp, tmd = dtm;
    int hit = dj >= 0 ? dj : HIT_NONE;
    int iters = 0;
    bool conv = true;

    // reduced-precision pencils not definite at p: decided by the FP64 pass
    if (bad && a.elist) {
        if (t == 0) a.elist[atomicAdd(a.ecount, 1)] = chain;
        return;
    }
    if (bad) st = SPEC_NOT_INTERIOR;
    if (!bad && m > 0) {
        const int kmax = a.kmax;
        double* Qg = a.Q + (size_t)chain * a.ldq;
        const LzLayout lz = lz_layout(scr, kmax);
        for (int dir = 0; dir < (a.both ? 2 : 1) && st == SPEC_OK; ++dir) {
            const double sg = dir == 0 ? 1.0 : -1.0;
            const bool vec_dir = a.want_vec && dir == 0;
            double tau = 0.0, tau_prev = 0.0, root = INFINITY;
            bool vec_ok = false, backoff = false, done = false;
            int rung = 0, halvings = 0;
            for (int it = 0; it < 210; ++it) {
                ++iters;
                fill_quadratic(L, Q0, Q1, Q2, tau, sg, P, t, blockDim.x);
                lds_barrier();
                const bool ok = chol_blocked(L, m, scr, sflag);
                lds_barrier();
                if (!ok) {
                    if (it == 0 && dir == 0 && a.elist) {
                        if (t == 0) a.elist[atomicAdd(a.ecount, 1)] = chain;
                        return;
                    }
                    if (it == 0) {
                        st = SPEC_NOT_INTERIOR;
                        done = true;
                        break;
                    }
                    // a step above the rounding level that left the feasible set:
                    // its bound was not a lower bound of lambda_min (single-vector
                    // Lanczos can converge to the second of two nearly equal smallest
                    // eigenvalues, as where two faces of S meet).  Halve it back
                    // towards the last definite iterate and step again from there.
                    if (!backoff && tau - tau_prev > 1e-12 * tau && halvings < 60) {
                        ++halvings;
                        tau = tau_prev + 0.5 * (tau - tau_prev);
                        continue;
                    }
                    // definiteness lost at the rounding level: the root is tau.  For the
                    // kernel vector, factor just inside it: root (1 - delta) for delta =
                    // 1e-12, 1e-10, 1e-8, 1e-6 (never below the last certified iterate)
                    // until a factor exists; there the pencil's most negative
                    // eigenvalue is isolated and its eigenvector is the kernel direction.
                    if (!backoff) root = tau;
                    if (!vec_dir || rung == 4) {  // no factor next to the root: no kernel vector
                        done = true;
                        break;
                    }
                    backoff = true;
                    const double delta = rung == 0 ? 1e-12 : (rung == 1 ? 1e-10 : (rung == 2 ? 1e-8 : 1e-6));
                    ++rung;
                    tau = fmax(root * (1.0 - delta), tau_prev);
                    continue;
                }
                tri_inverse(L, m, scr);
                // reduced-precision pencils of an ill-conditioned F(p): queued for
                // an FP64 assembly, which writes this chain's results
                if (it == 0 && dir == 0 && a.elist) {
                    const double pr = pivot_ratio(L, m, rtp);
                    if (pr < a.esc_ratio) {
                        if (t == 0) a.elist[atomicAdd(a.ecount, 1)] = chain;
                        return;
                    }
                }
                // lambda_min of D2, then of D1 (its basis stays for the kernel vector)
                double d[2] = {0.0, 0.0};
                for (int pass = backoff ? 1 : 0; pass < 2; ++pass) {
                    LzCtx lc;
                    lc.m = m;
                    lc.kmax = kmax;
                    lc.min_only = 1;
                    lc.first_check = 0;
                    // only a lower bound of lambda_min enters the step: theta - r is a
                    // bound at any tolerance, a looser one just shortens the step.  D1
                    // fixes the root and the kernel vector, so it is solved more tightly.
                    lc.tol = pass == 0 ? fmax(a.tol, 1e-3) : fmax(a.tol, 1e-6);
                    lc.loose_ratio = 0.0;
                    lc.tol_loose = 0.0;
                    lc.B0 = pass == 0 ? Q2 : Q1;
                    lc.b0 = pass == 0 ? 1.0 : sg;
                    lc.B1 = pass == 0 ? nullptr : Q2;
                    lc.b1 = pass == 0 ? 0.0 : 2.0 * tau;
                    lc.Qg = Qg;
                    lc.prof = nullptr;
                    lanczos_extreme(L, scr, lc);
                    __syncthreads();
                    if (pass == 1 && lz.sres[4] != 1.0) conv = false;
                    d[pass] = lz.sres[0] - lz.sres[1];
                    lds_barrier();
                }
                if (backoff) {
                    vec_ok = true;
                    done = true;
                    break;
                }
                const double step = first_root_q(d[1], d[0]);
                if (!(step < INFINITY)) {
                    done = true;
                    break;
                }
                const double next = tau + step;
                if (next > hz) {
                    done = true;
                    break;
                }
                if (step <= 1e-15 * next) {
                    root = next;
                    vec_ok = true;
                    done = true;
                    break;
                }
                tau_prev = tau;
                tau = next;
            }
            if (!done) {
                // out of iterations: the last definite iterate bounds the root
                // from below (no kernel vector there)
                conv = false;
                if (!backoff) root = tau_prev;
            }
            if (st != SPEC_OK) break;
            if (dir == 0) {
                if (root <= tp) {
                    tp = root;
                    hit = HIT_DENSE;
                    if (a.want_vec && vec_ok) {
                        __syncthreads();  // basis rows in HBM are read across lanes
                        const double lam = lz.sres[0];
                        ritz_u(L, scr, m, kmax, (int)lz.sres[5], lam, Qg, a.u + (size_t)chain * a.ldu,
                               a.U2 + (size_t)chain * a.ldu2);
                    } else if (a.want_vec) {
                        // no factor at the last iterate: no kernel vector (zero normal)
                        for (int e = t; e < P; e += blockDim.x) a.U2[(size_t)chain * a.ldu2 + e] = 0.0;
                    }
                }
            } else {
                tmd = fmin(tmd, root);
            }
            lds_barrier();
        }
    }
    // a hit from reduced-precision pencils: the reflection point and normal
    // need the FP64 root (the FP64 pass writes this chain's results)
    if (a.elist && st == SPEC_OK && isfinite(tp) && tp <= hz) {
        if (t == 0) a.elist[atomicAdd(a.ecount, 1)] = chain;
        return;
    }
    if (t == 0) {
        double tm = -tmd;
        if (st == SPEC_NOT_INTERIOR) {
            tm = NAN;
            tp = NAN;
            hit = HIT_NONE;
        } else if (!conv) {
            st = SPEC_NOCONV;
        }
        if (!a.both && st != SPEC_NOT_INTERIOR) tm = NAN;
        a.tm[chain] = tm;
        a.tp[chain] = tp;
        a.hit[chain] = isfinite(tp) ? hit : HIT_NONE;
        a.status[chain] = st;
        if (a.iters) a.iters[chain] = iters;
        if (a.flags) a.flags[chain] = a.idx ? SPEC_FLAG_ESCALATED : 0;
    }
}

// ---- degree-d curves (the polynomial eigenvalue problem of eq. (PEP))

constexpr int CURVE_DMAX = 6;

__device__ __forceinline__ double binom_small(int j, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (j - k + i) / i;
    return r;
}

// Smallest s > 0 with 1 + sum_{k=1..d} min(c_k, 0) s^k = 0 (+inf if every
// c_k >= 0): a decreasing function of s, so the root is bracketed by doubling
// and bisected to the last representable step.
__device__ inline double first_root_lower(const double* c, int d) {
    bool neg = false;
    for (int k = 1; k <= d; ++k) neg |= c[k] < 0.0;
    if (!neg) return INFINITY;
    auto g = [&](double s) {
        double v = 0.0;
        for (int k = d; k >= 1; --k) v = (v + fmin(c[k], 0.0)) * s;
        return 1.0 + v;
    };
    double hi = 1.0;
    while (g(hi) > 0.0 && hi < 1e300) hi *= 2.0;
    double lo = 0.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (g(mid) > 0.0) lo = mid; else hi = mid;
    }
    return lo;
}

// First positive root of q(t) = sum_k q_k t^k with q_0 > 0, not beyond hz:
// at tau, q(tau + s) / q(tau) = 1 + sum_k c_k s^k (Taylor coefficients over
// q(tau)) stays positive up to the root of the lower bound above; step there
// until the step is at the rounding level.
__device__ inline double poly_first_root(const double* q, int d, double hz) {
    double tau = 0.0;
    for (int it = 0; it < 400; ++it) {
        double c[CURVE_DMAX + 1];
        for (int k = 0; k <= d; ++k) {
            double v = 0.0;
            for (int j = d; j >= k; --j) v = v * tau + binom_small(j, k) * q[j];
            c[k] = v;
        }
        if (!(c[0] > 0.0)) return tau;
        for (int k = 1; k <= d; ++k) c[k] /= c[0];
        const double step = first_root_lower(c, d);
        if (!(step < INFINITY)) return INFINITY;
        const double next = tau + step;
        if (next > hz) return INFINITY;
        if (step <= 1e-15 * next) return next;
        tau = next;
    }
    return tau;
}

// F of the curve at tau: L = sum_k (sg tau)^k Q_k (Horner), packed.
__device__ inline void fill_poly(double* L, const double* const* Qk, int d, double tau, double sg, int P, int t,
                                 int bd) {
    const double x = sg * tau;
    for (int e = t; e < P; e += bd) {
        double v = Qk[d][e];
        for (int k = d - 1; k >= 0; --k) v = v * x + Qk[k][e];
        L[e] = v;
    }
}

// One workgroup per curve, the shape of k_curve2.  Dense block: at tau with
// Q(tau) = L L^T, L^-1 Q(tau + s) L^-T = I + sum_k s^k D_k with
// D_k = L^-1 (sum_{j >= k} C(j, k) tau^(j-k) Q_j) L^-T; by Weyl's inequality the
// pencil stays definite while 1 + sum_k s^k lambda_min(D_k) > 0, and
// 1 + sum_k min(d_k, 0) s^k with d_k = Ritz value minus residual bound is a
// lower bound of it, decreasing in s.  Each combination is written to the
// curve's scratch row and its lambda_min taken by Lanczos.  Steps that leave
// S are halved back as in k_curve2.  Diagonal rows: scalar polynomials.
__global__ __launch_bounds__(512) void k_curve_poly(CurveArgs a) {
    extern __shared__ double lds[];
    const int m = a.m, P = a.P, md = a.md, d = a.degree;
    const int row = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6, nw = blockDim.x >> 6;
    double* L = lds;
    double* scr = lds + P;
    int* sflag = (int*)(scr + 256);
    double* rtp = scr + 264;
    double* rtm = rtp + 8;
    int* rj = (int*)(rtm + 8);
    int* rbad = rj + 8;
    const double* Qk[CURVE_DMAX + 1];
    for (int k = 0; k <= d; ++k) Qk[k] = a.FB + ((size_t)k * a.brow0 + row) * a.ldfb;
    double* comb = a.comb + (size_t)row * a.ldfb;
    const double hz = a.horizon ? a.horizon[row] : a.hscalar;
    int32_t st = SPEC_OK;

    // ---- diagonal rows
    double dtp = INFINITY, dtm = INFINITY;
    int dj = -1, bad = 0;
    for (int j = t; j < md; j += blockDim.x) {
        double q[CURVE_DMAX + 1], qm[CURVE_DMAX + 1];
        for (int k = 0; k <= d; ++k) {
            q[k] = Qk[k][P + j];
            qm[k] = (k & 1) ? -q[k] : q[k];
        }
        if (!(q[0] > 0.0)) {
            bad = 1;
            continue;
        }
        const double sp = poly_first_root(q, d, hz);
        if (sp <= hz && sp < dtp) { dtp = sp; dj = j; }
        if (a.both) dtm = fmin(dtm, poly_first_root(qm, d, hz));
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double otp = __shfl_xor(dtp, o, 64);
        const int oj = __shfl_xor(dj, o, 64);
        if (otp < dtp || (otp == dtp && oj >= 0 && (dj < 0 || oj < dj))) { dtp = otp; dj = oj; }
        dtm = fmin(dtm, __shfl_xor(dtm, o, 64));
        bad |= __shfl_xor(bad, o, 64);
    }
    if (lane == 0) { rtp[wv] = dtp; rtm[wv] = dtm; rj[wv] = dj; rbad[wv] = bad; }
    lds_barrier();
    dtp = INFINITY; dtm = INFINITY; dj = -1; bad = 0;
    for (int w = 0; w < nw; ++w) {
        if (rtp[w] < dtp || (rtp[w] == dtp && rj[w] >= 0 && (dj < 0 || rj[w] < dj))) { dtp = rtp[w]; dj = rj[w]; }
        dtm = fmin(dtm, rtm[w]);
        bad |= rbad[w];
    }
    lds_barrier();
    double tp = dtp, tmd = dtm;
    int hit = dj >= 0 ? dj : HIT_NONE;
    int iters = 0;
    bool conv = true;
    if (bad) st = SPEC_NOT_INTERIOR;
    if (!bad && m > 0) {
        const int kmax = a.kmax;
        double* Qg = a.Q + (size_t)row * a.ldq;
        const LzLayout lz = lz_layout(scr, kmax);
        for (int dir = 0; dir < (a.both ? 2 : 1) && st == SPEC_OK; ++dir) {
            const double sg = dir == 0 ? 1.0 : -1.0;
            double tau = 0.0, tau_prev = 0.0, root = INFINITY;
            bool done = false;
            int halvings = 0;
            for (int it = 0; it < 400; ++it) {
                ++iters;
                fill_poly(L, Qk, d, tau, sg, P, t, blockDim.x);
                lds_barrier();
                const bool ok = chol_blocked(L, m, scr, sflag);
                lds_barrier();
                if (!ok) {
                    if (it == 0) {
                        st = SPEC_NOT_INTERIOR;
                        done = true;
                        break;
                    }
                    if (tau - tau_prev > 1e-12 * tau && halvings < 60) {
                        ++halvings;
                        tau = tau_prev + 0.5 * (tau - tau_prev);
                        continue;
                    }
                    root = tau;  // definiteness lost at the rounding level
                    done = true;
                    break;
                }
                tri_inverse(L, m, scr);
                double dk[CURVE_DMAX + 1];
                dk[0] = 1.0;
                for (int k = 1; k <= d; ++k) {
                    // Taylor coefficient sum_{j >= k} C(j, k) tau^(j-k) sg^j Q_j into the scratch row
                    for (int e = t; e < P; e += blockDim.x) {
                        double v = 0.0;
                        for (int j = d; j >= k; --j) v = v * tau + binom_small(j, k) * ((j & 1) ? sg : 1.0) * Qk[j][e];
                        comb[e] = v;
                    }
                    __syncthreads();  // the row is read back by the whole workgroup
                    LzCtx lc;
                    lc.m = m;
                    lc.kmax = kmax;
                    lc.min_only = 1;
                    lc.first_check = 0;
                    lc.tol = k == 1 ? fmax(a.tol, 1e-6) : fmax(a.tol, 1e-3);
                    lc.loose_ratio = 0.0;
                    lc.tol_loose = 0.0;
                    lc.B0 = comb;
                    lc.b0 = 1.0;
                    lc.B1 = nullptr;
                    lc.b1 = 0.0;
                    lc.Qg = Qg;
                    lc.prof = nullptr;
                    lanczos_extreme(L, scr, lc);
                    __syncthreads();
                    if (k == 1 && lz.sres[4] != 1.0) conv = false;
                    dk[k] = lz.sres[0] - lz.sres[1];
                    lds_barrier();
                }
                const double step = first_root_lower(dk, d);
                if (!(step < INFINITY)) {
                    done = true;
                    break;
                }
                const double next = tau + step;
                if (next > hz) {
                    done = true;
                    break;
                }
                if (step <= 1e-15 * next) {
                    root = next;
                    done = true;
                    break;
                }
                tau_prev = tau;
                tau = next;
            }
            if (!done) {
                conv = false;
                root = tau_prev;
            }
            if (dir == 0) {
                if (root <= tp) {
                    tp = root;
                    hit = HIT_DENSE;
                }
            } else {
                tmd = fmin(tmd, root);
            }
            lds_barrier();
        }
    }
    if (t == 0) {
        double tm = -tmd;
        if (st == SPEC_NOT_INTERIOR) {
            tm = NAN;
            tp = NAN;
            hit = HIT_NONE;
        } else if (!conv) {
            st = SPEC_NOCONV;
        }
        if (!a.both && st != SPEC_NOT_INTERIOR) tm = NAN;
        a.tm[row] = tm;
        a.tp[row] = tp;
        a.hit[row] = isfinite(tp) ? hit : HIT_NONE;
        a.status[row] = st;
        if (a.iters) a.iters[row] = iters;
        if (a.flags) a.flags[row] = 0;
    }
}

hipError_t launch_curve_poly(const CurveArgs& a, int nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    if (a.degree < 3 || a.degree > CURVE_DMAX || !a.comb) return hipErrorInvalidValue;
    const size_t lds = fused_lds_bytes(a.m, a.kmax);
    if (lds > 163840 || a.m > 2 * MAXH) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_curve_poly, dim3(nblocks), dim3(fused_threads(a.m)), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_curve2(const CurveArgs& a, int nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    const size_t lds = fused_lds_bytes(a.m, a.kmax);
    if (lds > 163840 || a.m > 2 * MAXH) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_curve2, dim3(nblocks), dim3(fused_threads(a.m)), lds, s, a);
    return hipGetLastError();
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

hipError_t launch_zero_ints(int* p, int count, hipStream_t s) {
    if (count <= 0 || count > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, s, p, count);
    return hipGetLastError();
}

int line_refine_blocks_per_cu(int max_m, int kmax) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_line_refine<false>),
                                                     fused_threads(max_m), fused_lds_bytes(max_m, kmax)) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu;
}

hipError_t launch_line_refine(const FusedArgs& one, const FusedArgs* args, const int2* work, const int* nwork,
                              int* counter, int max_m, int kmax, int nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    if (max_m > 2 * MAXH) return hipErrorInvalidValue;
    const size_t lds = fused_lds_bytes(max_m, kmax);
    if (lds > 163840) return hipErrorInvalidValue;
    if (args)
        hipLaunchKernelGGL(k_line_refine<true>, dim3(nblocks), dim3(fused_threads(max_m)), lds, s, one, args, work,
                           nwork, counter);
    else
        hipLaunchKernelGGL(k_line_refine<false>, dim3(nblocks), dim3(fused_threads(max_m)), lds, s, one, args, work,
                           nwork, counter);
    return hipGetLastError();
}

hipError_t launch_line_certify(const FusedArgs& a, int nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    if (a.m > 2 * MAXH) return hipErrorInvalidValue;
    const size_t lds = fused_lds_bytes(a.m, a.kmax);
    if (lds > 163840) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_line_certify, dim3(nblocks), dim3(fused_threads(a.m)), lds, s, a);
    return hipGetLastError();
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
