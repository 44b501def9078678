// Launch interfaces of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spec.h"

namespace spec {

// Which block attains t+ : a diagonal row index (>= 0), the dense block, or none.
enum : int { HIT_DENSE = -1, HIT_NONE = -3 };

hipError_t gemm_f64(bool transB, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
                    double* C, int ldc, hipStream_t s);
hipError_t mfma_probe(double* out, hipStream_t s);

size_t factor_lds_bytes(int m);
hipError_t launch_factor(int batch, int m, int md, int P, const double* FB, int ldfb, double* W, int ldw,
                         int32_t* status, hipStream_t s);

struct LanczosArgs {
    int batch, m, md, P, kmax;
    double tol;
    const double* FB;  // rows 0..batch-1: F(x_c); rows brow0 + c: B(v_c); ld ldfb
    int ldfb, brow0;
    const double* W;   // per chain packed L^{-1}, ld ldw
    int ldw;
    int32_t* status;   // in: factor status; out: final status
    double* tm;
    double* tp;
    int32_t* hit;      // row index (>= 0), HIT_DENSE, HIT_NONE
    double* lam;       // nullable: (lambda_min, lambda_max, lambda_2, iterations) per chain
    int want_vec;
    const double* ell; // nullable: the vector is only formed when t+ < ell[c]
    double* u;         // per chain kernel vector u (m), ld ldu
    int ldu;
    double* U2;        // per chain packed vec(u u^T) with doubled off-diagonal, ld ldu2
    int ldu2;
};
size_t lanczos_lds_bytes(int m, int kmax);
hipError_t launch_lanczos(const LanczosArgs& a, hipStream_t s);

// Assembly rows: Z[c] = [1, x_c] (F) and Z[zrow0 + c] = [0, v_c] (B), padded with zeros.
hipError_t launch_build_z(int batch, int n, int Kpad, const double* x, const double* v, double* Z, int zrow0,
                          hipStream_t s);

struct ReflectArgs {
    int batch, n, m, P, md, ldA;
    const double* Astk;  // (rows) x ldA; row i+1 = A_i packed, diagonal part at column P
    const int32_t* hit;
    const double* tp;
    const double* v;     // direction (batch x n)
    const double* wn;    // normal GEMM output (batch x ldwn)
    int ldwn;
    const double* lam;   // lambda_min, lambda_max, lambda_2 per chain (nullable)
    int32_t* status;
    double* s_out;       // reflected direction
    double* w_out;       // unit outward normal (nullable)
};
hipError_t launch_reflect_finish(const ReflectArgs& a, hipStream_t s);
hipError_t launch_sum_col(int rows, const double* M, int ld, int col, double* out, hipStream_t s);
hipError_t launch_status_to_flag(int batch, const int32_t* st, int8_t* flag, hipStream_t s);

}  // namespace spec
