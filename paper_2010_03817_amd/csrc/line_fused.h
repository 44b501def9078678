// Fused per-chain line oracle (internal launch interface).
#pragma once
#include "spec_kernels.h"

namespace spec {

struct FusedArgs {
    int m, md, P, kmax;
    double tol;
    const double* FB;          // row c: F(x_c) packed + diagonal rows; row brow0 + c: B(v_c)
    int ldfb, brow0;
    const int32_t* idx;        // nullable: workgroup b handles chain idx[b]
    const double* shift;       // nullable: per-chain origin t0 (learned bracket, lower end)
    const double* shift_hi;    // nullable: per-chain upper end, must not be definite
    int min_only;              // stop on lambda_min alone
    int first_check;           // step of the first convergence test (0: 4)
    int membership_only;       // Cholesky of F(x) only; status OK / NOT_INTERIOR
    int want_vec;              // form u and vec(u u^T) for dense hits
    const double* ell;         // nullable: only when t+ < ell[c]
    double* Q;                 // per chain Lanczos basis (kmax x m), ld ldq
    size_t ldq;
    int32_t* status;
    double* tm;
    double* tp;
    int32_t* hit;
    double* lam;               // nullable: (lambda_min, lambda_max, cert, steps) per chain
    double* u;
    int ldu;
    double* U2;
    int ldu2;
    long long* prof;           // nullable: per chain 8 clock64 stamps of the phases
    // far-root refinement (see line_fused_chain): a first-pass run from the
    // plain origin with rho > refine_ratio |lambda| for a deciding root stops
    // that side at tol_loose and queues (inst_id, chain) in rlist (count in
    // *rcount) with the origin rshift[chain] for the REFINE pass, whose
    // FusedArgs have shift = rshift
    double refine_ratio;       // 0: off
    double tol_loose;
    int2* rlist;               // nullable: no refinement
    int* rcount;
    double* rshift;
    int inst_id;
    int32_t* flags;            // nullable: per chain SPEC_FLAG_* bits
    double* cert;              // nullable: per chain the certified interval of t+ (2 doubles)
    // precision escalation (reduced-precision pencils): a chain whose factor at
    // the plain origin has min pivot / max pivot < esc_ratio is queued in elist
    // (count *ecount) without results; `escalated` marks the FP64 pass over them
    int32_t* elist;            // nullable: no escalation
    int* ecount;
    double esc_ratio;
    int escalated;
    // F(x) carried over from the previous round of a line walk (first pass
    // only): F(x_c) = upd_F[c] + s upd_B[c] with s = upd_s[c], the chain's move
    // along its previous direction (x_c = x_prev + s v_prev), written to FB's
    // row c for the later passes; s NaN: the chain was moved off that line
    // (back to its step start) and waits for the next full assembly (status
    // WALK_STALE, nothing else written).  Null: FB's F rows are current.
    const double* upd_F;
    const double* upd_B;
    const double* upd_s;
};

// Degree-2 curve oracle: first root of det Q(t), Q(t) = Q0 + t Q1 + t^2 Q2,
// by certified Weyl stepping (internal launch interface).
struct CurveArgs {
    int m, md, P, kmax;
    double tol;
    const double* FB;          // rows c, brow0 + c, 2 brow0 + c: Q0, Q1, Q2 of chain c (packed + diagonal rows)
    int ldfb, brow0;
    const double* horizon;     // nullable: per-chain horizon (else hscalar)
    double hscalar;
    int both;                  // also the first negative root (t-)
    int want_vec;              // form u and vec(u u^T) at a dense hit of the positive root
    double* Q;                 // per chain Lanczos basis (kmax x m), ld ldq
    size_t ldq;
    int32_t* status;
    double* tm;
    double* tp;
    int32_t* hit;              // HIT_DENSE, a diagonal row, or HIT_NONE
    int32_t* iters;            // nullable: Weyl steps (both directions)
    double* u;
    int ldu;
    double* U2;
    int ldu2;
    // precision escalation as FusedArgs; idx (nullable): workgroup j handles
    // chain idx[j] with pencil rows j (a compacted FP64 assembly)
    int32_t* elist;
    int* ecount;
    double esc_ratio;
    const int32_t* idx;
    int32_t* flags;            // nullable: SPEC_FLAG_ESCALATED set on the FP64 pass
    // degree >= 3 (launch_curve_poly): rows k brow0 + c, k = 0 .. degree, hold
    // Q_k; comb rows c (ld ldfb) are per-curve scratch for the Taylor
    // coefficients of the pencil
    int degree;
    double* comb;
};
hipError_t launch_curve2(const CurveArgs& a, int nblocks, hipStream_t s);
// First roots of det Q(t), Q(t) = sum_k t^k Q_k, for 3 <= degree <= 6
// (certified Taylor-Weyl stepping; no kernel vector).
hipError_t launch_curve_poly(const CurveArgs& a, int nblocks, hipStream_t s);

// Persistent launch over (instance, chain) items of several spectrahedra:
// args[instance] as for launch_line_fused, work[i] = (instance, chain) in the
// order items are to start, counter: one device int (reset by the launch),
// LDS sized for max_m and kmax (the largest over the instances).
hipError_t launch_line_fused_multi(const FusedArgs* args, const int2* work, int nwork, int* counter, int max_m,
                                   int kmax, int nblocks, hipStream_t s);

// Workgroups of the persistent launch resident per compute unit.
int line_fused_multi_blocks_per_cu(int max_m, int kmax);

// The REFINE pass: persistent workgroups over the queued items (count read
// on the device); args (per instance) or `one` when args is null.
hipError_t launch_line_refine(const FusedArgs& one, const FusedArgs* args, const int2* work, const int* nwork,
                              int* counter, int max_m, int kmax, int nblocks, hipStream_t s);
int line_refine_blocks_per_cu(int max_m, int kmax);
// p[0 .. count) = 0 by a kernel (no memset node in a captured graph); count <= 64.
hipError_t launch_zero_ints(int* p, int count, hipStream_t s);

// Two-sided Cholesky certificate of the dense t+ of each chain after the
// oracle passes (sets SPEC_FLAG_CHOL_CERT_FAILED on failure).
hipError_t launch_line_certify(const FusedArgs& a, int nblocks, hipStream_t s);

size_t fused_lds_bytes(int m, int kmax);
int fused_threads(int m);
hipError_t launch_line_fused(const FusedArgs& a, int nblocks, hipStream_t s);

}  // namespace spec
