// Host-side helpers shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "spec.h"

namespace spec_host {

inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

template <class T>
hipError_t dalloc(T** p, size_t count, bool zero = true) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * count);
    if (e != hipSuccess) return e;
    if (zero) e = hipMemset(*p, 0, sizeof(T) * count);
    return e;
}

template <class T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

inline spec_status from_hip(hipError_t e) {
    if (e == hipSuccess) return SPEC_OK;
    if (e == hipErrorOutOfMemory) return SPEC_ENOMEM;
    return SPEC_EDEVICE;
}

#define HIPCHK(expr)                                   \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return from_hip(_e);     \
    } while (0)
#define SPCHK(expr)                                    \
    do {                                               \
        spec_status _s = (expr);                       \
        if (_s != SPEC_OK) return _s;                  \
    } while (0)

}  // namespace spec_host

using namespace spec_host;
