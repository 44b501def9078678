// spec_intersect_noalloc_dev: spec_intersect_dev for callers that cannot
// allocate device memory (work under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).  The call's scratch (coefficient rows,
// assembled pencils, Lanczos bases, per-chain results of the first pass,
// the refinement queue) lives in one file-scope device array, `scratch`, of
// SPEC_NOALLOC_SCRATCH_BYTES; every call on a device shares that device's
// copy, which keeps the last call's contents.  Its device address comes from
// hipGetSymbolAddress, once per device, and only that address reaches the
// kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "abi_handle.h"
#include "mlp.h"
#include "spec_diag.h"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[SPEC_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on each device (the host-side name is not one).
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

spec_status scratch_on(int device, unsigned char** out) {
    if (device < 0 || device >= kMaxDevices) return SPEC_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return SPEC_EDEVICE;
        if (cur != device && hipSetDevice(device) != hipSuccess) return SPEC_EDEVICE;
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return SPEC_EDEVICE;
        g_scratch[device] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch[device]);
    return SPEC_OK;
}

// Carve consecutive 256-byte aligned pieces out of the scratch array (base 0:
// offsets only, to size a call).
struct Carver {
    uintptr_t base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + off);
        off += (sizeof(T) * count + 255) / 256 * 256;
        return p;
    }
};

struct Layout {
    double *Z, *FB, *Q, *Lam, *RShift;
    float* Z32;
    int32_t *Hit, *Flags;
    int2* RList;
    int* RCnt;
    size_t bytes;
};

Layout layout(const spec_s* h, int bp, uintptr_t base) {
    Carver c{base};
    Layout L{};
    L.Z = c.take<double>((size_t)2 * bp * h->Kpad);
    L.Z32 = c.take<float>(h->prec ? (size_t)2 * bp * h->Kpad : 0);
    L.FB = c.take<double>((size_t)2 * bp * h->ldA);
    L.Q = c.take<double>((size_t)bp * h->ldq());
    L.Lam = c.take<double>((size_t)bp * 4);
    L.RShift = c.take<double>((size_t)bp);
    L.Hit = c.take<int32_t>((size_t)bp);
    L.Flags = c.take<int32_t>((size_t)bp);
    L.RList = c.take<int2>((size_t)bp);
    L.RCnt = c.take<int>(2);
    L.bytes = c.off;
    return L;
}

}  // namespace

extern "C" {

spec_status spec_intersect_noalloc_dev(spec_handle h, int batch, const double* x, const double* v, double* t_minus,
                                       double* t_plus, int32_t* status, void* stream) {
    if (!h || batch < 0 || (batch && (!x || !v || !t_minus || !t_plus || !status))) return SPEC_EINVAL;
    if (batch == 0) return SPEC_OK;
    unsigned char* base = nullptr;
    SPCHK(scratch_on(h->device, &base));
    const int bp = round_up(batch, 64);
    // sizes only (base = null): the call is refused before any work
    if (layout(h, bp, 0).bytes > (size_t)SPEC_NOALLOC_SCRATCH_BYTES) return SPEC_ENOTSUP;
    const Layout L = layout(h, bp, reinterpret_cast<uintptr_t>(base));
    hipStream_t s = (hipStream_t)stream;
    // pencils F(x_c) (rows c) and B(v_c) (rows bp + c), as spec_intersect_dev
    HIPCHK(launch_build_z(batch, h->n, h->Kpad, x, v, L.Z, bp, s));
    const int M = 2 * bp;
    if (h->prec == 0) {
        HIPCHK(gemm_f64(false, M, h->ldA, h->Kpad, L.Z, h->Kpad, h->dA, h->ldA, L.FB, h->ldA, s));
    } else {
        HIPCHK(to_f32((size_t)M * h->Kpad, L.Z, L.Z32, s));
        HIPCHK(gemm_asm(h->prec - 1, M, h->ldA, h->Kpad, L.Z32, h->Kpad, h->dA32, h->ldA, L.FB, h->ldA, s));
    }
    FusedArgs a{};
    a.m = h->m;
    a.md = h->md;
    a.P = h->P;
    a.kmax = h->kmax;
    a.tol = h->tol;
    a.FB = L.FB;
    a.ldfb = h->ldA;
    a.brow0 = bp;
    a.Q = L.Q;
    a.ldq = h->ldq();
    a.status = status;
    a.tm = t_minus;
    a.tp = t_plus;
    a.hit = L.Hit;
    a.lam = L.Lam;
    a.refine_ratio = h->m > 0 ? h->refine_ratio : 0.0;
    a.tol_loose = h->tol_loose;
    a.rlist = a.refine_ratio > 0.0 ? L.RList : nullptr;
    a.rcount = L.RCnt;
    a.rshift = L.RShift;
    a.flags = L.Flags;
    if (!a.rlist) {
        HIPCHK(launch_line_fused(a, batch, s));
        return SPEC_OK;
    }
    // the queue counters start at zero in every call (a kernel, no memset)
    HIPCHK(launch_zero_ints(L.RCnt, 2, s));
    HIPCHK(launch_line_fused(a, batch, s));
    FusedArgs r = a;
    r.shift = L.RShift;
    r.rlist = nullptr;
    if (h->refine_bpc == 0) h->refine_bpc = line_refine_blocks_per_cu(h->m, h->kmax);
    const int nb = std::min(batch, h->refine_bpc * h->cus);
    HIPCHK(launch_line_refine(r, nullptr, L.RList, L.RCnt, L.RCnt + 1, h->m, h->kmax, nb, s));
    return SPEC_OK;
}

}  // extern "C"
