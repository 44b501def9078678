// The handle behind spec_handle (internal to the library): the instance's
// device copies, settings, workspace and walk state.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "spec.h"
#include "spec_kernels.h"
#include "walk_kernels.h"
#include "line_fused.h"
#include "mlp_net.h"
#include "abi_util.h"

using namespace spec;

struct spec_s {
    int device = 0;
    int n = 0, m = 0, md = 0, P = 0, Ptot = 0, K = 0, Kpad = 0, ldA = 0, Arows = 0, Nn = 0;
    double* dA = nullptr;  // Arows x ldA
    // pencil assembly precision: 0 FP64, 1 FP32 MFMA, 2 BF16 hi+lo MFMA (FP32 accumulation)
    int prec = 0;
    float* dA32 = nullptr;  // FP32 copy of the A-stack when prec > 0
    // Lanczos settings
    int kmax = 80;
    double tol = 1e-8;
    // refinement of far roots from a shifted origin (spec_options)
    double refine_ratio = 1e3, tol_loose = 1e-3;
    int certify = 0;  // 1: two-sided Cholesky certificate of every dense t+ (spec_options)
    double esc_ratio = 1e-3;  // reduced-precision pencils: FP64 again below this pivot ratio
    // line walks: F(x) assembled from x every `refresh` rounds and carried
    // over as F + s B(v) in between (1: assembled every round)
    int refresh = 16;
    // workspace (capacity in chains, multiple of 64); work_gen changes whenever
    // it is (re)allocated, so that cached device pointers can be revalidated
    int cap = 0;
    unsigned work_gen = 0;
    double *dZ = nullptr, *dFB = nullptr, *dQ = nullptr, *dU = nullptr, *dU2 = nullptr, *dWn = nullptr;
    float* dZ32 = nullptr;
    double *dLam = nullptr, *dTm = nullptr, *dTp = nullptr;
    // carried-over F(x): the other [F; B] block of the walk rounds (2 cap rows,
    // on first use) and the chains' moves
    double *dFB2 = nullptr, *dUpdS = nullptr;
    int fb2_cap = 0;
    int32_t *dHit = nullptr, *dSt = nullptr, *dFlags = nullptr;
    double* dCert = nullptr;  // certified interval of t+ per chain (2 doubles)
    // precision escalation: queued chains, count, compact coefficient rows
    int32_t* dEList = nullptr;
    int* dECnt = nullptr;
    double* dZc = nullptr;
    // far-root refinement queue: items, origins, counters (queued, taken)
    int2* dRList = nullptr;
    double* dRShift = nullptr;
    int* dRCnt = nullptr;
    int cus = 256, refine_bpc = 0;
    // staging for the host-pointer entry points
    int scap = 0;
    double *sX = nullptr, *sV = nullptr, *sO1 = nullptr, *sO2 = nullptr, *sS = nullptr, *sW = nullptr;
    int32_t* sSt = nullptr;
    int8_t* sI = nullptr;
    // stage timing
    bool timing = false;
    hipEvent_t ev[6] = {};
    double stage_ms[5] = {0, 0, 0, 0, 0}, stage_n[5] = {0, 0, 0, 0, 0}, lanczos_steps = 0;
    double asm_rows = 0;  // pencil rows assembled by the timed walk rounds
    double* dLamSum = nullptr;
    long long* dProf = nullptr;
    int prof_cap = 0;
    // learned bracket (attached network, half-width, mode) and its per-chain shifts
    spec_mlp_s* net = nullptr;
    double mdelta = 0.0;
    int lmode = 0;
    double *dShift = nullptr, *dShiftHi = nullptr, *dPred = nullptr, *dHz = nullptr;
    // walk state
    int wcap = 0;
    double *wX = nullptr, *wXs = nullptr, *wV = nullptr, *wEll = nullptr, *wStats = nullptr, *wSum = nullptr;
    int32_t *wNref = nullptr, *wActive = nullptr, *wCount = nullptr;
    long long* wStep = nullptr;
    // saved walk state (spec_walk_state)
    int scap_w = 0;
    double *vX = nullptr, *vXs = nullptr, *vV = nullptr, *vEll = nullptr, *vStats = nullptr;
    int32_t *vNref = nullptr, *vActive = nullptr;
    long long* vStep = nullptr;

    // degree >= 3 curves: coefficient rows ((d + 1) per curve) and pencils
    // ((d + 1) per curve plus a scratch row), sized on first use
    double *dZp = nullptr, *dFBp = nullptr;
    size_t pz_rows = 0, pf_rows = 0;
    spec_status ensure_poly(size_t zrows, size_t frows) {
        if (zrows > pz_rows) {
            dfree(dZp);
            pz_rows = 0;
            HIPCHK(dalloc(&dZp, zrows * Kpad));
            pz_rows = zrows;
        }
        if (frows > pf_rows) {
            dfree(dFBp);
            pf_rows = 0;
            HIPCHK(dalloc(&dFBp, frows * ldA, false));
            pf_rows = frows;
        }
        return SPEC_OK;
    }
    void free_work() {
        dfree(dZp); dfree(dFBp);
        pz_rows = pf_rows = 0;
        dfree(dZ); dfree(dZ32); dfree(dFB); dfree(dQ); dfree(dU); dfree(dU2); dfree(dWn);
        dfree(dFB2); dfree(dUpdS);
        fb2_cap = 0;
        dfree(dLam); dfree(dTm); dfree(dTp); dfree(dHit); dfree(dSt); dfree(dFlags);
        dfree(dRList); dfree(dRShift); dfree(dRCnt); dfree(dCert);
        dfree(dEList); dfree(dECnt); dfree(dZc);
        dfree(dShift); dfree(dShiftHi); dfree(dPred); dfree(dHz);
        cap = 0;
        ++work_gen;
    }
    void free_walk() {
        dfree(wX); dfree(wXs); dfree(wV); dfree(wEll); dfree(wStats); dfree(wSum);
        dfree(wNref); dfree(wActive); dfree(wCount); dfree(wStep);
        wcap = 0;
        free_saved();
    }
    void free_saved() {
        dfree(vX); dfree(vXs); dfree(vV); dfree(vEll); dfree(vStats); dfree(vNref); dfree(vActive); dfree(vStep);
        scap_w = 0;
    }
    spec_status ensure_walk(int chains) {
        if (chains <= wcap) return SPEC_OK;
        free_walk();
        const int c = round_up(chains, 64);
        HIPCHK(dalloc(&wX, (size_t)c * n, false));
        HIPCHK(dalloc(&wXs, (size_t)c * n, false));
        HIPCHK(dalloc(&wV, (size_t)c * n, false));
        HIPCHK(dalloc(&wEll, (size_t)c, false));
        HIPCHK(dalloc(&wStats, (size_t)c * WALK_NSTAT, false));
        HIPCHK(dalloc(&wSum, (size_t)WALK_NSTAT, false));
        HIPCHK(dalloc(&wNref, (size_t)c, false));
        HIPCHK(dalloc(&wActive, (size_t)c, false));
        HIPCHK(dalloc(&wCount, (size_t)1, false));
        HIPCHK(dalloc(&wStep, (size_t)c, false));
        wcap = c;
        return SPEC_OK;
    }
    void free_stage() {
        dfree(sX); dfree(sV); dfree(sO1); dfree(sO2); dfree(sS); dfree(sW); dfree(sSt); dfree(sI);
        scap = 0;
    }
    spec_status ensure(int batch) {
        if (batch <= cap) return SPEC_OK;
        free_work();
        const int c = round_up(batch, 64);
        HIPCHK(dalloc(&dZ, (size_t)3 * c * Kpad));
        HIPCHK(dalloc(&dZ32, (size_t)3 * c * Kpad));
        HIPCHK(dalloc(&dFB, (size_t)3 * c * ldA, false));
        HIPCHK(dalloc(&dQ, (size_t)c * ldq(), false));
        HIPCHK(dalloc(&dU, (size_t)c * m, false));
        HIPCHK(dalloc(&dU2, (size_t)c * ldA));
        HIPCHK(dalloc(&dWn, (size_t)c * Nn, false));
        HIPCHK(dalloc(&dLam, (size_t)c * 4));
        HIPCHK(dalloc(&dTm, (size_t)c));
        HIPCHK(dalloc(&dTp, (size_t)c));
        HIPCHK(dalloc(&dHit, (size_t)c));
        HIPCHK(dalloc(&dSt, (size_t)c));
        HIPCHK(dalloc(&dFlags, (size_t)c));
        HIPCHK(dalloc(&dRList, (size_t)c, false));
        HIPCHK(dalloc(&dRShift, (size_t)c));
        HIPCHK(dalloc(&dRCnt, (size_t)2));
        HIPCHK(dalloc(&dCert, (size_t)2 * c));
        HIPCHK(dalloc(&dEList, (size_t)c));
        HIPCHK(dalloc(&dECnt, (size_t)1));
        HIPCHK(dalloc(&dZc, (size_t)3 * c * Kpad));
        HIPCHK(dalloc(&dShift, (size_t)c));
        HIPCHK(dalloc(&dShiftHi, (size_t)c));
        HIPCHK(dalloc(&dPred, (size_t)c));
        HIPCHK(dalloc(&dHz, (size_t)c));
        HIPCHK(dalloc(&dUpdS, (size_t)c));
        cap = c;
        return SPEC_OK;
    }
    spec_status ensure_fb2() {
        if (dFB2 && fb2_cap == cap) return SPEC_OK;
        dfree(dFB2);
        fb2_cap = 0;
        HIPCHK(dalloc(&dFB2, (size_t)2 * cap * ldA, false));
        fb2_cap = cap;
        return SPEC_OK;
    }
    size_t ldq() const { return (size_t)kmax * std::max(m, 1); }
    spec_status ensure_stage(int batch) {
        if (batch <= scap) return SPEC_OK;
        free_stage();
        const int c = round_up(batch, 64);
        HIPCHK(dalloc(&sX, (size_t)c * n, false));
        HIPCHK(dalloc(&sV, (size_t)c * n, false));
        HIPCHK(dalloc(&sO1, (size_t)c, false));
        HIPCHK(dalloc(&sO2, (size_t)c, false));
        HIPCHK(dalloc(&sS, (size_t)c * n, false));
        HIPCHK(dalloc(&sW, (size_t)c * n, false));
        HIPCHK(dalloc(&sSt, (size_t)c, false));
        HIPCHK(dalloc(&sI, (size_t)c, false));
        scap = c;
        return SPEC_OK;
    }
};
