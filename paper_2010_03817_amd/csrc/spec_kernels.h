// Launch interfaces of the HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spec.h"

namespace spec {

// Which block attains t+ : a diagonal row index (>= 0), the dense block, or none.
enum : int { HIT_DENSE = -1, HIT_NONE = -3 };

// Status of a walk chain's oracle call skipped for want of F(x): the chain was
// moved off its line in the previous round and waits for the next full
// assembly of F (walk rounds that carry F over; never returned by the ABI).
constexpr int32_t WALK_STALE = 100;

// Per-call bits of the line oracle: the learned bracket was not certified
// (plain origin used), a far root was refined from a shifted origin, a
// refining factor did not exist (the run from 0 was repeated at the full
// tolerance), t+ is attained by two pieces of the boundary at once (two
// diagonal rows, or a diagonal row and the dense block, with equal roots: the
// normal is not determined there).
// UNCERTIFIED: the a posteriori interval of a dense t+ is wider than 2e-9 t+
// (or there is none); CHOL_CERT_FAILED: the optional Cholesky factor at the
// interval's lower end did not exist.
enum : int {
    SPEC_FLAG_CERT_FALLBACK = 1,
    SPEC_FLAG_REFINED = 4,
    SPEC_FLAG_REFINE_FAILED = 8,
    SPEC_FLAG_TIE = 16,
    SPEC_FLAG_UNCERTIFIED = 32,
    SPEC_FLAG_CHOL_CERT_FAILED = 64,
    SPEC_FLAG_ESCALATED = 128  // reduced-precision pencils redone in FP64 (ill-conditioned F)
};

hipError_t gemm_f64(bool transB, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
                    double* C, int ldc, hipStream_t s);
// One product of a grouped launch: C = A B (B not transposed; M, N multiples
// of 128, K of 16), its 128 x 128 tiles numbered from tile0 (products in
// increasing tile0, consecutive).
struct GemmItem {
    const double* A;
    const double* B;
    double* C;
    int lda, ldb, ldc, M, N, K, tile0;
};
// `count` products (d: device array), `items` tiles in all, in one launch;
// each tile bit for bit as gemm_f64 computes it.
hipError_t gemm_f64_grouped(const GemmItem* d, int count, int items, hipStream_t s);
hipError_t mfma_probe(double* out, hipStream_t s);

// Assembly rows: Z[c] = [1, x_c] (F) and Z[zrow0 + c] = [0, v_c] (B), padded with zeros;
// rows batch <= c < zrow0 of both halves are zero (zrow0 >= batch).
// Coefficient rows of one spectrahedron of a batch for launch_build_z_multi.
struct ZRows {
    int n, Kpad;
    const double* x;
    const double* v;
    double* Z;
};
hipError_t launch_build_z(int batch, int n, int Kpad, const double* x, const double* v, double* Z, int zrow0,
                          hipStream_t s);
// launch_build_z of `count` spectrahedra (d: device array) in one launch.
hipError_t launch_build_z_multi(const ZRows* d, int count, int batch, int zrow0, hipStream_t s);

// Compact copy of the coefficient rows of the chains in list[0 .. count):
// rows k * zc0 + j of Zc = rows k * z0 + list[j] of Z, k < nrows; the rows
// count .. zc0 - 1 of each group are zero.
hipError_t launch_gather_rows(int count, int zc0, int nrows, int Kpad, const int32_t* list, const double* Z, int z0,
                              double* Zc, hipStream_t s);

// Rows k * zrow0 + c, k = 0, 1, 2, of Z: coefficient rows of curve c
// (nrows of them given, the rest zero), zero-padded to Kpad.
hipError_t launch_build_z_coef(int batch, int n, int Kpad, int nrows, const double* coef, double* Z, int zrow0,
                               hipStream_t s);
// All nrows coefficient rows of each curve: row k of curve c at k * zrow0 + c.
hipError_t launch_build_z_rows(int batch, int n, int Kpad, int nrows, const double* coef, double* Z, int zrow0,
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
    const int32_t* flags;  // nullable: SPEC_FLAG_* bits of the line oracle call
    int32_t* status;
    double* s_out;       // reflected direction
    double* w_out;       // unit outward normal (nullable)
};
hipError_t launch_reflect_finish(const ReflectArgs& a, hipStream_t s);
hipError_t launch_sum_col(int rows, const double* M, int ld, int col, double* out, hipStream_t s);
hipError_t launch_status_to_flag(int batch, const int32_t* st, int8_t* flag, hipStream_t s);

}  // namespace spec
