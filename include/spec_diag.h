/*
 * spec_diag.h -- diagnostic entry points of the spectrahedron oracle library
 * (checks of the device building blocks; not part of the method).
 * Host pointers; synchronous; return spec_status.
 */
#ifndef SPEC_DIAG_H
#define SPEC_DIAG_H
#include "spec.h"
#ifdef __cplusplus
extern "C" {
#endif

/* Runs one v_mfma_f64_16x16x4f64 on a wave with A[i][k] in lane i + 16 k and
 * B[k][j] in lane j + 16 k, A[i][0] = 1, A[i][1] = i, B[0][j] = 1000 j,
 * B[1][j] = 1 (else 0), so D[i][j] = 1000 j + i; host_out receives the
 * 64 lanes x 4 accumulator doubles (256 values). */
spec_status spec_diag_mfma_layout(double* host_out);

/* C = A * B (transB = 0: B is K x N) or A * B^T (transB = 1: B is N x K),
 * all row-major float64 host arrays; M, N multiples of 64, K of 16 (also
 * N = 208 with transB = 1: the narrow kernel of the boundary normal). */
spec_status spec_diag_gemm_f64(int transB, int M, int N, int K, const double* A, const double* B, double* C);

/* After an intersect/reflect call of `batch` elements: per element
 * (lambda_min(C), lambda_max(C) of the last Lanczos run, learned-bracket code
 * (0: none or certified, 1: lower end not certified, plain origin used,
 * 2: upper end definite in mode 2), Lanczos steps over every run). */
spec_status spec_diag_lanczos_info(spec_handle h, int batch, double* lam_out);

/* After an intersect/reflect call of `batch` elements: per element the bits
 * 1 (learned bracket not certified), 4 (a far root refined from a shifted
 * origin), 8 (the factor at that origin did not exist; plain solve at the
 * full tolerance). */
spec_status spec_diag_call_flags(spec_handle h, int batch, int32_t* flags_out);

/* Stage timing of the walk rounds, measured with HIP events recorded on the
 * walk's stream around each stage.  spec_diag_timing(h, 1) resets and turns
 * it on, (h, 0) turns it off.  spec_diag_stage_times writes, per stage
 * (0 assembly GEMM, 1 network prediction of the learned bracket, 2 fused
 * factor + Lanczos kernel, 3 normal GEMM, 4 walk update), the
 * summed milliseconds and the number of launches (2 x 5 doubles); also the
 * Lanczos step count summed over chains of the timed rounds (1 double). */
spec_status spec_diag_timing(spec_handle h, int on);
spec_status spec_diag_stage_times(spec_handle h, double* ms_and_counts, double* lanczos_steps);
/* Pencil rows (F(x) and B(v) rows, one per chain each) that the line-oracle
 * rounds assembled while timing was on: a round that carries F(x) over
 * assembles only the B(v) rows (spec_options.refresh_period). */
spec_status spec_diag_assembly_rows(spec_handle h, double* rows);

/* Phase stamps of the per-chain kernel: spec_diag_phase_profile(h, c)
 * records, for the next calls on chains < c, SPEC_DIAG_PHASE_SLOTS values
 * per chain: the shader clock (clock64) of thread 0 at 7 phase boundaries
 * (slots 0..6: start, F loaded, Cholesky, inverse, Lanczos start, Lanczos
 * end, done); the Cholesky's diagonal-tile, panel and trailing-update cycles
 * (slots 7, 14, 15); the cycles the steering wave spent in the parts of the
 * Lanczos steps (slots 8..13: q stored, W^T q, B a, W b and alpha, beta, stop
 * test and the closing barrier); the stop tests run and the Sturm passes
 * they made (slots 16, 17), and the cycles of their multisection and of
 * their residual bounds and decisions (slots 18, 19); the busy cycles of
 * wave 1 (trailing tiles and inverse rows) and of wave 0 (next diagonal
 * tile) in the Cholesky's trailing phases (slots 20, 23); the last inverse
 * row's product and store cycles (slots 21, 22).  0 turns it off.  spec_diag_phase_stamps copies
 * batch x SPEC_DIAG_PHASE_SLOTS values to the host.  Calls must use
 * batch <= c. */
#define SPEC_DIAG_PHASE_SLOTS 24
spec_status spec_diag_phase_profile(spec_handle h, int max_chains);
spec_status spec_diag_phase_stamps(spec_handle h, int batch, long long* out);

/* One MFMA instruction per trial (one wave each), operands given per lane:
 * kind 0 = v_mfma_f32_16x16x4f32 (a, b: trials x 64 floats), kind 1 =
 * v_mfma_f32_16x16x32_bf16 (a, b: trials x 64 x 8 floats, rounded to
 * bfloat16); d: trials x 64 x 4 accumulator registers.  Host pointers. */
spec_status spec_diag_mfma_raw(int kind, int trials, const float* a, const float* b, float* d);

/* The MLP's GEMM on host buffers: C (M x ldc) = op(A) op(B) with op(A) M x K
 * (ta: A stored K x M), op(B) K x N (tb: B stored N x K), bf16 operands when
 * bf16 != 0, epilogue mode 0 store, 1 C = Z and aux = GELU(Z), 2 C = acc *
 * GELU'(aux).  aux is M x ldaux (read and/or written), nullable for mode 0. */
spec_status spec_diag_gemm_f32(int ta, int tb, int bf16, int mode, int M, int N, int K, const float* A, int lda,
                               const float* B, int ldb, float* C, int ldc, float* aux, int ldaux);

#ifdef __cplusplus
}
#endif
#endif
