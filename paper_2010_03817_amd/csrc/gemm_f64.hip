// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64), used for the
// two contractions of the oracle that are shared by every chain:
//   pencil assembly   [F(x); B(v)] = [1 x; 0 v] * Astack      (B not transposed)
//   boundary normal   w = vec(u u^T) * Astack^T                (B transposed)
// (paper: construction of the pencil in O(n m^2), Lemma "intersection cost";
//  normal (u^T A_i u)_i in O(n m^2), Lemma "reflection cost").
//
// Tiling: a 256-thread workgroup computes a 128x128 tile of C when M and N
// allow it (see k_gemm_f64_128), else a 64x64 tile, each of its four waves a
// 32x32 quarter as 2x2 MFMA 16x16 blocks.  K advances 16 at a time through
// LDS.  M, N, K must be multiples of 64, 64, 16 (callers pad with zeros).
// Workgroups are ordered so that the eight XCDs each walk their own
// contiguous range of N tiles: a B panel is then fetched into one XCD's L2
// and reused there by every M tile.
#include "common.h"
#include "spec_kernels.h"

namespace spec {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GT_M = 64, GT_N = 64, GT_K = 16;
constexpr int LDA_S = GT_K + 1;   // padded LDS row of the A tile (bank spread)
constexpr int LDB_S = GT_N + 2;

template <bool TRANS_B>
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int N, int K, const double* __restrict__ A,
                                                  int lda, const double* __restrict__ B, int ldb,
                                                  double* __restrict__ C, int ldc) {
    __shared__ double As[GT_M * LDA_S];
    __shared__ double Bs[GT_K * LDB_S];

    const int tilesM = M / GT_M, tilesN = N / GT_N;
    // XCD-aware order: hardware places workgroup g on XCD g % 8.  Give XCD x the
    // tiles [x*T/8, (x+1)*T/8) in M-fastest order.
    const int total = tilesM * tilesN;
    const int g = blockIdx.x;
    int lin;
    if (total % 8 == 0) {
        const int per = total / 8;
        lin = (g % 8) * per + g / 8;
    } else {
        lin = g;
    }
    const int tm = lin % tilesM, tn = lin / tilesM;
    const int row0 = tm * GT_M, col0 = tn * GT_N;

    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < K; k0 += GT_K) {
        // A tile: 64 x 16
        {
            const int r = t >> 2, c = (t & 3) * 4;
            const double* src = A + (size_t)(row0 + r) * lda + k0 + c;
#pragma unroll
            for (int q = 0; q < 4; ++q) As[r * LDA_S + c + q] = src[q];
        }
        if (!TRANS_B) {
            const int r = t >> 4, c = (t & 15) * 4;
            const double* src = B + (size_t)(k0 + r) * ldb + col0 + c;
#pragma unroll
            for (int q = 0; q < 4; ++q) Bs[r * LDB_S + c + q] = src[q];
        } else {
            // B is N x K row-major: Bs[k][n] = B[col0 + n][k0 + k]
            const int nn = t >> 2, kk = (t & 3) * 4;
            const double* src = B + (size_t)(col0 + nn) * ldb + k0 + kk;
#pragma unroll
            for (int q = 0; q < 4; ++q) Bs[(kk + q) * LDB_S + nn] = src[q];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < GT_K; ks += 4) {
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[(wr + i * 16 + (lane & 15)) * LDA_S + ks + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[(ks + (lane >> 4)) * LDB_S + wc + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulator r of lane l holds D[l/16 + 4 r][l % 16] of its 16x16 block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = row0 + wr + i * 16 + (lane >> 4) + 4 * r;
                const int cc = col0 + wc + j * 16 + (lane & 15);
                // streaming store: the output is not read again by this kernel
                __builtin_nontemporal_store(acc[i][j][r], &C[(size_t)rr * ldc + cc]);
            }
}

// 128 x 128 tiles for shapes that allow them: each wave computes a 64 x 64
// quarter as 4 x 4 MFMA blocks (half the operand traffic per flop of the
// 64 x 64 tiling), the LDS stage is double-buffered and the next K slice is
// read from global memory into registers while the current one is multiplied,
// so that one barrier per K step suffices: buffer (s+1) mod 2 is written at
// step s only after the barrier that ends step s-1, the last reads of it.
constexpr int BT = 128, BK = 16;
constexpr int LAS = BK + 1;   // padded LDS rows (bank spread)
constexpr int LBS = BT + 2;

template <bool TRANS_B>
// Work items: every output tile once (ksplit = 1), or twice, for the two
// halves of the K slices (ksplit = 2), each half adding its partial tile into
// C, which the caller has zeroed: two additions onto zero give fl(a + b) in
// either order, so the result does not depend on which half lands first.
// Persistent: the gridDim.x workgroups (about two per CU) walk the items;
// when the items divide into eight ranges, workgroup g stays in range g % 8
// (its XCD under round-robin dispatch), and within a range the tiles go in
// groups of GROUP_M tile rows, the rows of a group fastest, so that the tiles
// in flight on one XCD share a few A row panels and B column panels (a
// working set that stays in that XCD's L2).  The first K slice of a
// workgroup's next item is read while the current tile is stored.
__global__ __launch_bounds__(256) void k_gemm_f64_128(int M, int N, int K, const double* __restrict__ A,
                                                      int lda, const double* __restrict__ B, int ldb,
                                                      double* __restrict__ C, int ldc, int ksplit) {
    __shared__ double As[2][BT * LAS];
    __shared__ double Bs[2][BK * LBS];

    const int tilesM = M / BT, tilesN = N / BT;
    const int total = tilesM * tilesN;
    const int items = total * ksplit;
    const int G = gridDim.x, g = blockIdx.x;
    const bool ranges = items % 8 == 0 && G % 8 == 0;
    const int per = items / 8, GX = G / 8;
    const int nks = K / BK, kmid = (nks / 2) * BK;
    constexpr int GROUP_M = 8;
    const int gsz = GROUP_M * tilesN;
    // the i-th item of this workgroup (-1 past the end)
    auto item_at = [&](int i) -> int {
        if (ranges) {
            const int j = g / 8 + GX * i;
            return j < per ? (g % 8) * per + j : -1;
        }
        const int it = g + G * i;
        return it < items ? it : -1;
    };
    struct Job {
        int row0, col0, kbeg, kend;
    };
    auto job_of = [&](int it) -> Job {
        const int part = it / total;  // K half (ksplit = 2), else 0
        const int lin = it - part * total;
        const int first_m = (lin / gsz) * GROUP_M;
        const int gm = tilesM - first_m < GROUP_M ? tilesM - first_m : GROUP_M;
        const int in_g = lin % gsz;
        Job jb;
        jb.row0 = (first_m + in_g % gm) * BT;
        jb.col0 = (in_g / gm) * BT;
        jb.kbeg = ksplit == 2 && part == 1 ? kmid : 0;
        jb.kend = ksplit == 2 && part == 0 ? kmid : K;
        return jb;
    };

    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr = (wv >> 1) * 64, wc = (wv & 1) * 64;
    // global -> LDS mapping of one K slice: 8 consecutive doubles per thread
    const int ar = t >> 1, ac = (t & 1) * 8;                          // A: row ar, columns ac..ac+7
    const int br = TRANS_B ? (t & 1) * 8 : t >> 4, bc = TRANS_B ? t >> 1 : (t & 15) * 8;
    double ra[8], rb[8];
    auto fetch = [&](int row0, int col0, int k0) {
        const double* pa = A + (size_t)(row0 + ar) * lda + k0 + ac;
#pragma unroll
        for (int q = 0; q < 8; ++q) ra[q] = pa[q];
        if (!TRANS_B) {
            const double* pb = B + (size_t)(k0 + br) * ldb + col0 + bc;
#pragma unroll
            for (int q = 0; q < 8; ++q) rb[q] = pb[q];
        } else {
            // B is N x K row-major: row col0 + bc, columns k0 + br ..
            const double* pb = B + (size_t)(col0 + bc) * ldb + k0 + br;
#pragma unroll
            for (int q = 0; q < 8; ++q) rb[q] = pb[q];
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 8; ++q) As[buf][ar * LAS + ac + q] = ra[q];
        if (!TRANS_B) {
#pragma unroll
            for (int q = 0; q < 8; ++q) Bs[buf][br * LBS + bc + q] = rb[q];
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) Bs[buf][(br + q) * LBS + bc] = rb[q];
        }
    };

    int it = item_at(0);
    if (it < 0) return;  // uniform over the workgroup
    Job jb = job_of(it);
    fetch(jb.row0, jb.col0, jb.kbeg);
    stash(0);
    __syncthreads();
    for (int i = 1;; ++i) {
        d4 acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        // slice s of this item is in LDS buffer s & 1 (slice 0 stashed above)
        for (int k0 = jb.kbeg, s = 0; k0 < jb.kend; k0 += BK, ++s) {
            const int cur = s & 1;
            const bool more = k0 + BK < jb.kend;
            if (more) fetch(jb.row0, jb.col0, k0 + BK);
            const double* as = As[cur];
            const double* bs = Bs[cur];
#pragma unroll
            for (int ks = 0; ks < BK; ks += 4) {
                double a[4], b[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) a[q] = as[(wr + q * 16 + (lane & 15)) * LAS + ks + (lane >> 4)];
#pragma unroll
                for (int q = 0; q < 4; ++q) b[q] = bs[(ks + (lane >> 4)) * LBS + wc + q * 16 + (lane & 15)];
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p][q], 0, 0, 0);
            }
            if (more) stash(cur ^ 1);
            __syncthreads();  // (the last one: every wave is done with both buffers)
        }
        // the next item's first slice, read while this tile is stored
        const int nit = item_at(i);
        Job nj{0, 0, 0, 0};
        if (nit >= 0) {
            nj = job_of(nit);
            fetch(nj.row0, nj.col0, nj.kbeg);
        }
        // accumulator r of lane l holds D[l/16 + 4 r][l % 16] of its 16x16 block
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = jb.row0 + wr + p * 16 + (lane >> 4) + 4 * r;
                    const int cc = jb.col0 + wc + q * 16 + (lane & 15);
                    double* pc = &C[(size_t)rr * ldc + cc];
                    if (ksplit == 2) unsafeAtomicAdd(pc, acc[p][q][r]);
                    // streaming store: the output is not read again by this kernel
                    else __builtin_nontemporal_store(acc[p][q][r], pc);
                }
        if (nit < 0) break;
        stash(0);
        __syncthreads();
        jb = nj;
    }
}

// A group of independent products C_k = A_k B_k (B not transposed) in one
// persistent launch: the 128 x 128 tiles of every product are items
// d[k].tile0 .. d[k].tile0 + tiles_k - 1 (tiles_k = M_k N_k / 128^2, M_k and
// N_k multiples of 128, K_k of 16), walked by the workgroups in steps of the
// grid; each tile is computed exactly as k_gemm_f64_128 computes it (the same
// K slices, LDS stage and MFMA order), so the results are bit for bit those
// of one launch per product.  For the many small assemblies of an uneven
// batch, whose launches would otherwise outnumber their work.
__global__ __launch_bounds__(256) void k_gemm_f64_128_grouped(const GemmItem* __restrict__ d, int count,
                                                              int items) {
    __shared__ double As[2][BT * LAS];
    __shared__ double Bs[2][BK * LBS];
    const int G = gridDim.x, g = blockIdx.x;
    struct Job {
        const double* A;
        const double* B;
        double* C;
        int lda, ldb, ldc, K, row0, col0;
    };
    auto job_of = [&](int it) -> Job {
        int lo = 0, hi = count - 1;  // the last product whose first item is <= it
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d[mid].tile0 <= it) lo = mid;
            else hi = mid - 1;
        }
        const GemmItem& q = d[lo];
        const int lin = it - q.tile0, tilesM = q.M / BT;
        return Job{q.A, q.B, q.C, q.lda, q.ldb, q.ldc, q.K, (lin % tilesM) * BT, (lin / tilesM) * BT};
    };
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int wr = (wv >> 1) * 64, wc = (wv & 1) * 64;
    const int ar = t >> 1, ac = (t & 1) * 8;
    const int br = t >> 4, bc = (t & 15) * 8;
    double ra[8], rb[8];
    auto fetch = [&](const Job& jb, int k0) {
        const double* pa = jb.A + (size_t)(jb.row0 + ar) * jb.lda + k0 + ac;
#pragma unroll
        for (int q = 0; q < 8; ++q) ra[q] = pa[q];
        const double* pb = jb.B + (size_t)(k0 + br) * jb.ldb + jb.col0 + bc;
#pragma unroll
        for (int q = 0; q < 8; ++q) rb[q] = pb[q];
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 8; ++q) As[buf][ar * LAS + ac + q] = ra[q];
#pragma unroll
        for (int q = 0; q < 8; ++q) Bs[buf][br * LBS + bc + q] = rb[q];
    };
    int it = g;
    if (it >= items) return;  // uniform over the workgroup
    Job jb = job_of(it);
    fetch(jb, 0);
    stash(0);
    __syncthreads();
    for (;;) {
        d4 acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0, s = 0; k0 < jb.K; k0 += BK, ++s) {
            const int cur = s & 1;
            const bool more = k0 + BK < jb.K;
            if (more) fetch(jb, k0 + BK);
            const double* as = As[cur];
            const double* bs = Bs[cur];
#pragma unroll
            for (int ks = 0; ks < BK; ks += 4) {
                double a[4], b[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) a[q] = as[(wr + q * 16 + (lane & 15)) * LAS + ks + (lane >> 4)];
#pragma unroll
                for (int q = 0; q < 4; ++q) b[q] = bs[(ks + (lane >> 4)) * LBS + wc + q * 16 + (lane & 15)];
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p][q], 0, 0, 0);
            }
            if (more) stash(cur ^ 1);
            __syncthreads();
        }
        const int nit = it + G;
        Job nj{};
        if (nit < items) {
            nj = job_of(nit);
            fetch(nj, 0);
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = jb.row0 + wr + p * 16 + (lane >> 4) + 4 * r;
                    const int cc = jb.col0 + wc + q * 16 + (lane & 15);
                    __builtin_nontemporal_store(acc[p][q][r], &jb.C[(size_t)rr * jb.ldc + cc]);
                }
        if (nit >= items) break;
        stash(0);
        __syncthreads();
        jb = nj;
        it = nit;
    }
}

// C = 0 by a kernel (no memset node when the launch is captured into a graph).
__global__ void k_zero_f64(double* __restrict__ C, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) C[i] = 0.0;
}

// Narrow transposed product C (M x 16 NB, ld ldc) = A (M x K) B^T, B given as
// 16 NB rows of length K (the normal w = vec(u u^T) Astack^T with n just
// above a multiple of 64: n = 200 takes 13 column blocks, 208 columns, where
// the 128-wide tiles would compute 256).  A workgroup of NW waves computes a
// 16 NW x 16 NB tile; wave w the rows 16 w .. 16 w + 15 against all NB column
// blocks, so each A operand feeds NB MFMAs.  K slices of 16 go through a double-buffered
// LDS stage as in k_gemm_f64_128 (the next slice read into registers while
// the current one is multiplied, one barrier per slice); items are the tiles,
// or their two K halves added into a zeroed C (ksplit = 2), walked by a
// persistent grid of about two workgroups per CU, workgroup g in the eighth
// of the items of its XCD (g mod 8).  M % (16 NW) == 0, K % 16 == 0.
constexpr int NLA = BK + 1;
template <int NB, int NW>
__global__ __launch_bounds__(64 * NW) void k_gemm_f64_nt_narrow(int M, int K, const double* __restrict__ A, int lda,
                                                                const double* __restrict__ B, int ldb,
                                                                double* __restrict__ C, int ldc, int ksplit) {
    constexpr int NC = 16 * NB, NLB = NC + 2, NM = 16 * NW;
    static_assert(NC <= 64 * NW, "one B row per thread");
    __shared__ double As[2][NM * NLA];
    __shared__ double Bs[2][BK * NLB];
    const int total = M / NM;
    const int items = total * ksplit;
    const int G = gridDim.x, g = blockIdx.x;
    const bool ranges = items % 8 == 0 && G % 8 == 0;
    const int per = items / 8, GX = G / 8;
    const int nks = K / BK, kmid = (nks / 2) * BK;
    auto item_at = [&](int i) -> int {
        if (ranges) {
            const int j = g / 8 + GX * i;
            return j < per ? (g % 8) * per + j : -1;
        }
        const int it = g + G * i;
        return it < items ? it : -1;
    };
    struct Job {
        int row0, kbeg, kend;
    };
    auto job_of = [&](int it) -> Job {
        const int part = it / total;
        Job jb;
        jb.row0 = (it - part * total) * NM;
        jb.kbeg = ksplit == 2 && part == 1 ? kmid : 0;
        jb.kend = ksplit == 2 && part == 0 ? kmid : K;
        return jb;
    };
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    // one K slice: A rows t / 4, four columns each; B row t (t < NC), 16 columns
    const int ar = t >> 2, ac = (t & 3) * 4;
    const bool bown = t < NC;
    double ra[4], rb[BK];
    auto fetch = [&](int row0, int k0) {
        const double* pa = A + (size_t)(row0 + ar) * lda + k0 + ac;
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[q] = pa[q];
        if (bown) {
            const double* pb = B + (size_t)t * ldb + k0;
#pragma unroll
            for (int q = 0; q < BK; ++q) rb[q] = pb[q];
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) As[buf][ar * NLA + ac + q] = ra[q];
        if (bown) {
#pragma unroll
            for (int q = 0; q < BK; ++q) Bs[buf][q * NLB + t] = rb[q];
        }
    };
    int it = item_at(0);
    if (it < 0) return;  // uniform over the workgroup
    Job jb = job_of(it);
    fetch(jb.row0, jb.kbeg);
    stash(0);
    __syncthreads();
    for (int i = 1;; ++i) {
        d4 acc[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
        for (int k0 = jb.kbeg, s = 0; k0 < jb.kend; k0 += BK, ++s) {
            const int cur = s & 1;
            const bool more = k0 + BK < jb.kend;
            if (more) fetch(jb.row0, k0 + BK);
            const double* as = As[cur];
            const double* bs = Bs[cur];
#pragma unroll
            for (int ks = 0; ks < BK; ks += 4) {
                const double a = as[(16 * wv + (lane & 15)) * NLA + ks + (lane >> 4)];
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    const double b = bs[(ks + (lane >> 4)) * NLB + 16 * q + (lane & 15)];
                    acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
                }
            }
            if (more) stash(cur ^ 1);
            __syncthreads();
        }
        const int nit = item_at(i);
        Job nj{0, 0, 0};
        if (nit >= 0) {
            nj = job_of(nit);
            fetch(nj.row0, nj.kbeg);
        }
        // accumulator r of lane l holds D[l/16 + 4 r][l % 16] of its 16x16 block
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = jb.row0 + 16 * wv + (lane >> 4) + 4 * r;
                double* pc = &C[(size_t)rr * ldc + 16 * q + (lane & 15)];
                if (ksplit == 2) unsafeAtomicAdd(pc, acc[q][r]);
                else __builtin_nontemporal_store(acc[q][r], pc);
            }
        if (nit < 0) break;
        stash(0);
        __syncthreads();
        jb = nj;
    }
}

static int cu_count() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

hipError_t gemm_f64(bool transB, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
                    double* C, int ldc, hipStream_t s) {
    if (transB && N == 208 && M % 64 == 0 && K % BK == 0 && ldc >= N) {
        if (M == 0) return hipSuccess;
        // the narrow transposed product (13 column blocks) in 64-row tiles, two
        // 4-wave workgroups per CU (128-row tiles of one 8-wave workgroup per
        // CU measured slower); two K halves per tile when the tiles are fewer
        // than the workgroups that fit
        const int cus = cu_count(), tiles = M / 64;
        const int ksplit = tiles < 2 * cus && K >= 4096 ? 2 : 1;
        if (ksplit == 2) {
            const size_t n = (size_t)M * ldc;
            hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, n);
        }
        const int items = tiles * ksplit;
        const int grid = items < 2 * cus ? items : 2 * cus;
        hipLaunchKernelGGL((k_gemm_f64_nt_narrow<13, 4>), dim3(grid), dim3(256), 0, s, M, K, A, lda, B, ldb, C, ldc,
                           ksplit);
        return hipGetLastError();
    }
    if (M % GT_M || N % GT_N || K % GT_K) return hipErrorInvalidValue;
    if (M == 0 || N == 0) return hipSuccess;
    if (M % BT == 0 && N % BT == 0) {
        const int tiles = (M / BT) * (N / BT);
        // fewer tiles than two per CU and a long K: two K halves per tile, so
        // that two workgroups share each CU (the output is zeroed first)
        const int ksplit = tiles < 512 && K >= 4096 ? 2 : 1;
        if (ksplit == 2) {
            const size_t n = (size_t)M * N;
            if (ldc != N) return hipErrorInvalidValue;
            hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, n);
        }
        // persistent grid: two workgroups per CU (LDS 68 KB each), at most one per item
        const int cus = cu_count();
        const int items = tiles * ksplit;
        const int grid = items < 2 * cus ? items : 2 * cus;
        if (transB)
            hipLaunchKernelGGL(k_gemm_f64_128<true>, dim3(grid), dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc,
                               ksplit);
        else
            hipLaunchKernelGGL(k_gemm_f64_128<false>, dim3(grid), dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc,
                               ksplit);
        return hipGetLastError();
    }
    const int tiles = (M / GT_M) * (N / GT_N);
    if (transB)
        hipLaunchKernelGGL(k_gemm_f64<true>, dim3(tiles), dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
    else
        hipLaunchKernelGGL(k_gemm_f64<false>, dim3(tiles), dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
    return hipGetLastError();
}

hipError_t gemm_f64_grouped(const GemmItem* d, int count, int items, hipStream_t s) {
    if (count <= 0 || items <= 0) return hipSuccess;
    const int cus = cu_count();
    const int grid = items < 2 * cus ? items : 2 * cus;
    hipLaunchKernelGGL(k_gemm_f64_128_grouped, dim3(grid), dim3(256), 0, s, d, count, items);
    return hipGetLastError();
}

// Probe of the MFMA lane layout: A(16x4) and B(4x16) given in the documented
// operand layout (lane l holds A[l%16][l/16] and B[l/16][l%16]) with
// A[i][0] = 1, A[i][1] = i, B[0][j] = 1000 j, B[1][j] = 1 and zeros elsewhere,
// so D[i][j] = 1000 j + i; every accumulator double of every lane is written.
__global__ void k_mfma_probe(double* out) {
    const int lane = threadIdx.x;
    const int ij = lane & 15, k = lane >> 4;
    const double a = k == 0 ? 1.0 : (k == 1 ? (double)ij : 0.0);
    const double b = k == 0 ? 1000.0 * ij : (k == 1 ? 1.0 : 0.0);
    d4 acc{0.0, 0.0, 0.0, 0.0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    for (int r = 0; r < 4; ++r) out[lane * 4 + r] = acc[r];
}

hipError_t mfma_probe(double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, s, out);
    return hipGetLastError();
}

}  // namespace spec
