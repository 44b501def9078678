// MLP kernels of the learned boundary bracket (internal launch interface).
//
// Parameters follow one packed FP32 layout: for each layer l, W_l (in_l x out_l,
// row-major) immediately followed by its bias b_l (out_l), so that [W_l; b_l]
// is an (in_l + 1) x out_l row-major block.  Activations carry a trailing
// column of ones (leading dimension >= in_l + 1), which turns every affine map
// into one GEMM with K = in_l + 1 and makes the bias gradient the last row of
// the weight-gradient GEMM.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spec {

enum GemmMode : int {
    GEMM_STORE = 0,     // C = acc
    GEMM_GELU = 1,      // C = acc (pre-activation Z), aux = GELU(Z)
    GEMM_GELU_BWD = 2,  // C = acc * GELU'(aux)  (aux holds Z)
};

// C[M x N] = op(A) op(B) (+ epilogue).  op(A) is M x K: A row-major M x K
// (ta = 0) or K x M (ta = 1).  op(B) is K x N: B row-major K x N (tb = 0) or
// N x K (tb = 1).  bf16 = 1 rounds both operands to bfloat16 (round to nearest
// even) and runs the BF16 MFMA; bf16 = 0 runs the FP32 MFMA.  Accumulation is
// FP32 in both.
hipError_t gemm_f32(bool ta, bool tb, bool bf16, int mode, int M, int N, int K, const float* A, int lda,
                    const float* B, int ldb, float* C, int ldc, float* aux, int ldaux, hipStream_t s);

// Reduced-precision pencil assembly: C (FP64, M x N) = A (M x K) B (K x N),
// FP32 row-major operands, FP32 accumulation; prec 0 FP32 MFMA, 1 BF16 hi+lo
// pairs (three BF16 MFMA products).
hipError_t gemm_asm(int prec, int M, int N, int K, const float* A, int lda, const float* B, int ldb, double* C, int ldc,
                    hipStream_t s);
hipError_t to_f32(size_t count, const double* x, float* y, hipStream_t s);

// Features [(x - mu_x) * isd_x, (v - mu_v) * isd_v, (products), 1] of rows (FP64 in, FP32 out,
// ldf >= 2n + nextra + 1).
// The two products of (x, v) that may follow them in the features: <x, v> and
// |x|^2 (rows x 2, FP64).
hipError_t mlp_products(int rows, int n, const double* x, int ldx, const double* v, int ldv, double* out,
                        hipStream_t s);
// nextra = 2 appends the standardised products <x, v>, |x|^2 before the ones column.
hipError_t mlp_features(int rows, int n, int nextra, const double* x, int ldx, const double* v, int ldv,
                        const float* mu,
                        const float* isd, float* F, int ldf, hipStream_t s);
// Standardised targets ((log t+ - mu0) * isd0, (log(-t-) - mu1) * isd1).
hipError_t mlp_targets(int rows, const double* tm, const double* tp, const float* tmu, const float* tisd,
                       float* T, hipStream_t s);
// Rows out[r] = src[idx[r]] (ld columns copied: cols).
hipError_t mlp_gather(int rows, int cols, const int32_t* idx, const float* src, int lds, float* dst, int ldd,
                      hipStream_t s);
// Uniform random row indices in [0, range) from Philox (key seed, counter (r, step)).
hipError_t mlp_sample_rows(int rows, int range, uint64_t seed, uint32_t step, int32_t* idx, hipStream_t s);
// delta = 2 (Y - T) / (rows * cols); loss += sum (Y - T)^2 (FP64 accumulator).
hipError_t mlp_mse(int rows, int cols, const float* Y, int ldy, const float* T, float* delta, double* loss,
                   hipStream_t s);
// Adam on FP32 master parameters.
hipError_t mlp_adam(int64_t np, float* p, const float* g, float* m, float* v, int step, float lr, float b1, float b2,
                    float eps, hipStream_t s);
// Parameter init: W ~ U(-1/sqrt(in), 1/sqrt(in)), b = 0; ones column of an activation buffer.
hipError_t mlp_init(int nl, const int* dims, float* params, uint64_t seed, hipStream_t s);
hipError_t mlp_fill_col(int rows, float* A, int ld, int col, float val, hipStream_t s);
// t_lo = exp(log t+_hat - delta), t_hi (nullable) = exp(log t+_hat + delta), FP64 per
// row; pred_out (nullable) keeps log t+_hat.  Y holds standardised outputs.
hipError_t mlp_shift(int rows, const float* Y, int ldy, float mu0, float sd0, double delta, double* t_lo,
                     double* t_hi, double* pred_out, hipStream_t s);
// Outputs back to log scale: o0 = Y0 sd0 + mu0, o1 = Y1 sd1 + mu1 (nullable each).
hipError_t mlp_unstandardise(int rows, const float* Y, int ldy, float mu0, float sd0, float mu1, float sd1, double* o0,
                             double* o1, hipStream_t s);
// D[r] = [X[r, 0..cols), 1].
hipError_t mlp_augment(int rows, int cols, const float* X, int ldx, float* D, int ldd, hipStream_t s);
// Column sums and sums of squares (FP64) of rows x cols FP64 data.
hipError_t mlp_col_moments(int rows, int cols, const double* X, int ldx, double* sum, double* sumsq, hipStream_t s);

// Lane-layout probes of one MFMA instruction: kind 0 = FP32 16x16x4 (1 value per
// lane and operand), kind 1 = BF16 16x16x32 (8 values).  trials independent waves.
hipError_t mfma_raw_probe(int kind, int trials, const float* a, const float* b, float* d, hipStream_t s);

}  // namespace spec
