// MLP of the learned boundary bracket: BF16 / FP32 MFMA GEMM with fused GELU
// epilogues, loss, Adam and the feature / shift kernels around it.
#include "mlp.h"

#include "common.h"

namespace spec {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, LDS_K = BK + 4;

__device__ __forceinline__ short bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// GELU with the exact normal CDF, and its derivative.
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// 64 x 64 output tile per workgroup of 4 waves; wave w owns the 32 x 32
// quadrant (w >> 1, w & 1) as 2 x 2 MFMA blocks of 16 x 16.  Accumulator
// register r of lane l is D[4 (l / 16) + r][l % 16] for both MFMA shapes.
template <bool TA, bool TB, bool BF16, int MODE>
__global__ __launch_bounds__(256) void k_gemm_f32(int M, int N, int K, const float* __restrict__ A, int lda,
                                                  const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                                  float* __restrict__ aux, int ldaux) {
    __shared__ float As[BM][LDS_K];
    __shared__ float Bs[BN][LDS_K];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int lr = lane & 15, lg = lane >> 4;
    f4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += BK) {
        for (int e = t; e < BM * BK; e += 256) {
            int mm, kk;
            if (!TA) { mm = e / BK; kk = e % BK; }
            else { mm = e % BM; kk = e / BM; }
            const int gm = m0 + mm, gk = k0 + kk;
            float val = 0.f;
            if (gm < M && gk < K) val = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
            As[mm][kk] = val;
        }
        for (int e = t; e < BN * BK; e += 256) {
            int nn, kk;
            if (TB) { nn = e / BK; kk = e % BK; }
            else { nn = e % BN; kk = e / BN; }
            const int gn = n0 + nn, gk = k0 + kk;
            float val = 0.f;
            if (gn < N && gk < K) val = TB ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
            Bs[nn][kk] = val;
        }
        __syncthreads();
        if (BF16) {
            short8 av[2], bv[2];
            for (int i = 0; i < 2; ++i)
                for (int q = 0; q < 8; ++q) {
                    av[i][q] = bf16_rne(As[wm + 16 * i + lr][8 * lg + q]);
                    bv[i][q] = bf16_rne(Bs[wn + 16 * i + lr][8 * lg + q]);
                }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[i]),
                                                                        __builtin_bit_cast(bf16x8, bv[j]),
                                                                        acc[i][j], 0, 0, 0);
        } else {
            for (int kq = 0; kq < BK; kq += 4) {
                float a0 = As[wm + lr][kq + lg], a1 = As[wm + 16 + lr][kq + lg];
                float b0 = Bs[wn + lr][kq + lg], b1 = Bs[wn + 16 + lr][kq + lg];
                acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * i + 4 * lg + r, gn = n0 + wn + 16 * j + lr;
                if (gm >= M || gn >= N) continue;
                const float z = acc[i][j][r];
                if (MODE == GEMM_STORE) {
                    C[(size_t)gm * ldc + gn] = z;
                } else if (MODE == GEMM_GELU) {
                    C[(size_t)gm * ldc + gn] = z;
                    aux[(size_t)gm * ldaux + gn] = gelu(z);
                } else {
                    C[(size_t)gm * ldc + gn] = z * gelu_d(aux[(size_t)gm * ldaux + gn]);
                }
            }
}

// Reduced-precision assembly of packed pencils: C (M x N, FP64 out) = A B with
// A (M x K) and B (K x N) row-major FP32.  PREC 0: FP32 MFMA; PREC 1: BF16
// hi+lo pairs, a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi (three BF16 MFMAs).
// FP32 accumulation in both.  Same 64 x 64 tiling as k_gemm_f32.
template <int PREC>
__global__ __launch_bounds__(256) void k_gemm_asm(int M, int N, int K, const float* __restrict__ A, int lda,
                                                  const float* __restrict__ B, int ldb, double* __restrict__ C,
                                                  int ldc) {
    __shared__ float As[BM][LDS_K];
    __shared__ float Bs[BN][LDS_K];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int lr = lane & 15, lg = lane >> 4;
    f4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += BK) {
        for (int e = t; e < BM * BK; e += 256) {
            const int mm = e / BK, kk = e % BK, gm = m0 + mm, gk = k0 + kk;
            As[mm][kk] = (gm < M && gk < K) ? A[(size_t)gm * lda + gk] : 0.f;
        }
        for (int e = t; e < BN * BK; e += 256) {
            const int nn = e % BN, kk = e / BN, gn = n0 + nn, gk = k0 + kk;
            Bs[nn][kk] = (gn < N && gk < K) ? B[(size_t)gk * ldb + gn] : 0.f;
        }
        __syncthreads();
        if (PREC == 1) {
            short8 ah[2], al[2], bh[2], bl[2];
            for (int i = 0; i < 2; ++i)
                for (int q = 0; q < 8; ++q) {
                    const float av = As[wm + 16 * i + lr][8 * lg + q], bv = Bs[wn + 16 * i + lr][8 * lg + q];
                    const short ahq = bf16_rne(av), bhq = bf16_rne(bv);
                    ah[i][q] = ahq;
                    bh[i][q] = bhq;
                    al[i][q] = bf16_rne(av - __uint_as_float((uint32_t)(uint16_t)ahq << 16));
                    bl[i][q] = bf16_rne(bv - __uint_as_float((uint32_t)(uint16_t)bhq << 16));
                }
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al[i]),
                                                                        __builtin_bit_cast(bf16x8, bh[j]),
                                                                        acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                                        __builtin_bit_cast(bf16x8, bl[j]),
                                                                        acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ah[i]),
                                                                        __builtin_bit_cast(bf16x8, bh[j]),
                                                                        acc[i][j], 0, 0, 0);
                }
        } else {
            for (int kq = 0; kq < BK; kq += 4) {
                const float a0 = As[wm + lr][kq + lg], a1 = As[wm + 16 + lr][kq + lg];
                const float b0 = Bs[wn + lr][kq + lg], b1 = Bs[wn + 16 + lr][kq + lg];
                acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + 16 * i + 4 * lg + r, gn = n0 + wn + 16 * j + lr;
                if (gm < M && gn < N) C[(size_t)gm * ldc + gn] = (double)acc[i][j][r];
            }
}

__global__ void k_to_f32(size_t count, const double* __restrict__ x, float* __restrict__ y) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) y[e] = (float)x[e];
}

template <bool TA, bool TB, bool BF16>
hipError_t gemm_mode(int mode, dim3 g, int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C,
                     int ldc, float* aux, int ldaux, hipStream_t s) {
    if (mode == GEMM_STORE)
        k_gemm_f32<TA, TB, BF16, GEMM_STORE><<<g, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux);
    else if (mode == GEMM_GELU)
        k_gemm_f32<TA, TB, BF16, GEMM_GELU><<<g, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux);
    else
        k_gemm_f32<TA, TB, BF16, GEMM_GELU_BWD><<<g, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux);
    return hipGetLastError();
}

// <x, v> and |x|^2 of row r in FP64 (128 threads: two waves).
__device__ inline void row_products(int n, const double* __restrict__ x, const double* __restrict__ v, double& xv,
                                    double& xx) {
    __shared__ double red[2][2];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        a += x[i] * v[i];
        b += x[i] * x[i];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = a;
        red[threadIdx.x >> 6][1] = b;
    }
    __syncthreads();
    xv = red[0][0] + red[1][0];
    xx = red[0][1] + red[1][1];
}

__global__ __launch_bounds__(128) void k_features(int rows, int n, int nextra, const double* __restrict__ x, int ldx,
                                                  const double* __restrict__ v, int ldv,
                                                  const float* __restrict__ mu, const float* __restrict__ isd,
                                                  float* __restrict__ F, int ldf) {
    const int r = blockIdx.x;
    if (r >= rows) return;
    float* f = F + (size_t)r * ldf;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        f[i] = ((float)x[(size_t)r * ldx + i] - mu[i]) * isd[i];
        f[n + i] = ((float)v[(size_t)r * ldv + i] - mu[n + i]) * isd[n + i];
    }
    if (nextra) {
        double xv, xx;
        row_products(n, x + (size_t)r * ldx, v + (size_t)r * ldv, xv, xx);
        if (threadIdx.x == 0) {
            f[2 * n] = ((float)xv - mu[2 * n]) * isd[2 * n];
            f[2 * n + 1] = ((float)xx - mu[2 * n + 1]) * isd[2 * n + 1];
        }
    }
    if (threadIdx.x == 0) f[2 * n + nextra] = 1.0f;
}

__global__ __launch_bounds__(128) void k_products(int rows, int n, const double* __restrict__ x, int ldx,
                                                  const double* __restrict__ v, int ldv, double* __restrict__ out) {
    const int r = blockIdx.x;
    if (r >= rows) return;
    double xv, xx;
    row_products(n, x + (size_t)r * ldx, v + (size_t)r * ldv, xv, xx);
    if (threadIdx.x == 0) {
        out[2 * r] = xv;
        out[2 * r + 1] = xx;
    }
}

__global__ void k_targets(int rows, const double* __restrict__ tm, const double* __restrict__ tp,
                          const float* __restrict__ tmu, const float* __restrict__ tisd, float* __restrict__ T) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    T[2 * r] = ((float)log(tp[r]) - tmu[0]) * tisd[0];
    T[2 * r + 1] = ((float)log(-tm[r]) - tmu[1]) * tisd[1];
}

__global__ void k_gather(int rows, int cols, const int32_t* __restrict__ idx, const float* __restrict__ src, int lds,
                         float* __restrict__ dst, int ldd) {
    const int r = blockIdx.x;
    if (r >= rows) return;
    const float* s = src + (size_t)idx[r] * lds;
    float* d = dst + (size_t)r * ldd;
    for (int c = threadIdx.x; c < cols; c += blockDim.x) d[c] = s[c];
}

__global__ void k_sample_rows(int rows, int range, uint64_t seed, uint32_t step, int32_t* __restrict__ idx) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    double a, b;
    draw_u2(seed, (uint32_t)r, step, 0, TAG_MLP_BATCH, a, b);
    int k = (int)(a * (double)range);
    idx[r] = k < range ? k : range - 1;
}

__global__ void k_mse(int rows, int cols, const float* __restrict__ Y, int ldy, const float* __restrict__ T,
                      float* __restrict__ delta, double* __restrict__ loss) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double sq = 0.0;
    if (e < rows * cols) {
        const int r = e / cols, c = e % cols;
        const float d = Y[(size_t)r * ldy + c] - T[e];
        delta[e] = 2.0f * d / (float)((double)rows * cols);
        sq = (double)d * d;
    }
    sq = wave_sum(sq);
    if ((threadIdx.x & 63) == 0 && loss) atomicAdd(loss, sq);
}

__global__ void k_adam(int64_t np, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_init(int64_t off, int rows_in, int out, float bound, uint64_t seed, float* __restrict__ p) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nw = (int64_t)rows_in * out;
    if (e >= nw + out) return;
    if (e >= nw) {
        p[off + e] = 0.0f;
        return;
    }
    double a, b;
    draw_u2(seed, (uint32_t)(off + e), 0, 0, TAG_MLP_INIT, a, b);
    p[off + e] = (float)((2.0 * a - 1.0) * bound);
}

__global__ void k_fill_col(int rows, float* __restrict__ A, int ld, int col, float val) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < rows) A[(size_t)r * ld + col] = val;
}

__global__ void k_shift(int rows, const float* __restrict__ Y, int ldy, float mu0, float sd0, double delta,
                        double* __restrict__ t_lo, double* __restrict__ t_hi, double* __restrict__ pred) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const double lt = (double)Y[(size_t)r * ldy] * sd0 + mu0;
    double tl = exp(lt - delta);
    if (!(tl > 0.0) || !isfinite(tl)) tl = 0.0;  // a useless prediction: plain origin
    t_lo[r] = tl;
    if (t_hi) t_hi[r] = exp(lt + delta);
    if (pred) pred[r] = lt;
}

__global__ void k_unstd(int rows, const float* __restrict__ Y, int ldy, float mu0, float sd0, float mu1, float sd1,
                        double* __restrict__ o0, double* __restrict__ o1) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    if (o0) o0[r] = (double)Y[(size_t)r * ldy] * sd0 + mu0;
    if (o1) o1[r] = (double)Y[(size_t)r * ldy + 1] * sd1 + mu1;
}

__global__ void k_augment(int rows, int cols, const float* __restrict__ X, int ldx, float* __restrict__ D, int ldd) {
    const int r = blockIdx.x;
    if (r >= rows) return;
    for (int c = threadIdx.x; c < cols; c += blockDim.x) D[(size_t)r * ldd + c] = X[(size_t)r * ldx + c];
    if (threadIdx.x == 0) D[(size_t)r * ldd + cols] = 1.0f;
}

__global__ void k_col_moments(int rows, int cols, const double* __restrict__ X, int ldx, double* __restrict__ sum,
                              double* __restrict__ sumsq) {
    // block: 64 columns (lanes) x 4 waves over a chunk of rows
    const int c = blockIdx.x * 64 + (threadIdx.x & 63);
    const int w = threadIdx.x >> 6;
    const int chunk = (rows + gridDim.y - 1) / gridDim.y;
    const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
    if (c >= cols) return;
    double s = 0.0, q = 0.0;
    for (int r = r0 + w; r < r1; r += 4) {
        const double x = X[(size_t)r * ldx + c];
        s += x;
        q += x * x;
    }
    atomicAdd(sum + c, s);
    atomicAdd(sumsq + c, q);
}

__global__ void k_mfma_raw(int kind, const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ d) {
    const int l = threadIdx.x, trial = blockIdx.x;
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    if (kind == 0) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[trial * 64 + l], b[trial * 64 + l], acc, 0, 0, 0);
    } else {
        short8 av, bv;
        for (int q = 0; q < 8; ++q) {
            av[q] = bf16_rne(a[(trial * 64 + l) * 8 + q]);
            bv[q] = bf16_rne(b[(trial * 64 + l) * 8 + q]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                      acc, 0, 0, 0);
    }
    for (int r = 0; r < 4; ++r) d[(trial * 64 + l) * 4 + r] = acc[r];
}

}  // namespace

hipError_t gemm_f32(bool ta, bool tb, bool bf16, int mode, int M, int N, int K, const float* A, int lda,
                    const float* B, int ldb, float* C, int ldc, float* aux, int ldaux, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const dim3 g((N + BN - 1) / BN, (M + BM - 1) / BM);
    const int key = (ta ? 4 : 0) | (tb ? 2 : 0) | (bf16 ? 1 : 0);
    switch (key) {
        case 0: return gemm_mode<false, false, false>(mode, g, M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux, s);
        case 1: return gemm_mode<false, false, true>(mode, g, M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux, s);
        case 2: return gemm_mode<false, true, false>(mode, g, M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux, s);
        case 3: return gemm_mode<false, true, true>(mode, g, M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux, s);
        case 4: return gemm_mode<true, false, false>(mode, g, M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux, s);
        case 5: return gemm_mode<true, false, true>(mode, g, M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux, s);
        case 6: return gemm_mode<true, true, false>(mode, g, M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux, s);
        default: return gemm_mode<true, true, true>(mode, g, M, N, K, A, lda, B, ldb, C, ldc, aux, ldaux, s);
    }
}

hipError_t gemm_asm(int prec, int M, int N, int K, const float* A, int lda, const float* B, int ldb, double* C, int ldc,
                    hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const dim3 g((N + BN - 1) / BN, (M + BM - 1) / BM);
    if (prec == 1) k_gemm_asm<1><<<g, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc);
    else k_gemm_asm<0><<<g, 256, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc);
    return hipGetLastError();
}

hipError_t to_f32(size_t count, const double* x, float* y, hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_to_f32<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(count, x, y);
    return hipGetLastError();
}

hipError_t mlp_features(int rows, int n, int nextra, const double* x, int ldx, const double* v, int ldv,
                        const float* mu, const float* isd, float* F, int ldf, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    if (nextra != 0 && nextra != 2) return hipErrorInvalidValue;
    k_features<<<rows, 128, 0, s>>>(rows, n, nextra, x, ldx, v, ldv, mu, isd, F, ldf);
    return hipGetLastError();
}

hipError_t mlp_products(int rows, int n, const double* x, int ldx, const double* v, int ldv, double* out,
                        hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_products<<<rows, 128, 0, s>>>(rows, n, x, ldx, v, ldv, out);
    return hipGetLastError();
}

hipError_t mlp_targets(int rows, const double* tm, const double* tp, const float* tmu, const float* tisd, float* T,
                       hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_targets<<<(rows + 255) / 256, 256, 0, s>>>(rows, tm, tp, tmu, tisd, T);
    return hipGetLastError();
}

hipError_t mlp_gather(int rows, int cols, const int32_t* idx, const float* src, int lds, float* dst, int ldd,
                      hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_gather<<<rows, 128, 0, s>>>(rows, cols, idx, src, lds, dst, ldd);
    return hipGetLastError();
}

hipError_t mlp_sample_rows(int rows, int range, uint64_t seed, uint32_t step, int32_t* idx, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_sample_rows<<<(rows + 255) / 256, 256, 0, s>>>(rows, range, seed, step, idx);
    return hipGetLastError();
}

hipError_t mlp_mse(int rows, int cols, const float* Y, int ldy, const float* T, float* delta, double* loss,
                   hipStream_t s) {
    const int ne = rows * cols;
    if (ne <= 0) return hipSuccess;
    k_mse<<<(ne + 255) / 256, 256, 0, s>>>(rows, cols, Y, ldy, T, delta, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(int64_t np, float* p, const float* g, float* m, float* v, int step, float lr, float b1, float b2,
                    float eps, hipStream_t s) {
    if (np <= 0) return hipSuccess;
    const float c1 = (float)(1.0 - pow((double)b1, step)), c2 = (float)(1.0 - pow((double)b2, step));
    k_adam<<<(unsigned)((np + 255) / 256), 256, 0, s>>>(np, p, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_init(int nl, const int* dims, float* params, uint64_t seed, hipStream_t s) {
    int64_t off = 0;
    for (int l = 0; l < nl; ++l) {
        const int64_t cnt = (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
        const float bound = 1.0f / sqrtf((float)dims[l]);
        k_init<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(off, dims[l], dims[l + 1], bound, seed, params);
        off += cnt;
    }
    return hipGetLastError();
}

hipError_t mlp_fill_col(int rows, float* A, int ld, int col, float val, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_fill_col<<<(rows + 255) / 256, 256, 0, s>>>(rows, A, ld, col, val);
    return hipGetLastError();
}

hipError_t mlp_shift(int rows, const float* Y, int ldy, float mu0, float sd0, double delta, double* t_lo,
                     double* t_hi, double* pred_out, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_shift<<<(rows + 255) / 256, 256, 0, s>>>(rows, Y, ldy, mu0, sd0, delta, t_lo, t_hi, pred_out);
    return hipGetLastError();
}

hipError_t mlp_unstandardise(int rows, const float* Y, int ldy, float mu0, float sd0, float mu1, float sd1, double* o0,
                             double* o1, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_unstd<<<(rows + 255) / 256, 256, 0, s>>>(rows, Y, ldy, mu0, sd0, mu1, sd1, o0, o1);
    return hipGetLastError();
}

hipError_t mlp_augment(int rows, int cols, const float* X, int ldx, float* D, int ldd, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    k_augment<<<rows, 128, 0, s>>>(rows, cols, X, ldx, D, ldd);
    return hipGetLastError();
}

hipError_t mlp_col_moments(int rows, int cols, const double* X, int ldx, double* sum, double* sumsq, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const int chunks = rows < 256 ? 1 : 256;
    k_col_moments<<<dim3((cols + 63) / 64, chunks), 256, 0, s>>>(rows, cols, X, ldx, sum, sumsq);
    return hipGetLastError();
}

hipError_t mfma_raw_probe(int kind, int trials, const float* a, const float* b, float* d, hipStream_t s) {
    if (trials <= 0) return hipSuccess;
    k_mfma_raw<<<trials, 64, 0, s>>>(kind, a, b, d);
    return hipGetLastError();
}

}  // namespace spec
