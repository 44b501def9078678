// Small per-chain kernels around the oracle: assembly rows and the
// reflection of eq. (reflection).
#include "common.h"
#include "spec_kernels.h"

namespace spec {

// Rows c < batch as above; rows batch <= c < zrow0 of both halves are zero
// (the padding rows of the GEMM: defined whatever the buffer held before).
__device__ __forceinline__ void build_z_row(int c, int batch, int n, int Kpad, const double* __restrict__ x,
                                            const double* __restrict__ v, double* __restrict__ Z, int zrow0) {
    double* zf = Z + (size_t)c * Kpad;
    double* zb = Z + (size_t)(zrow0 + c) * Kpad;
    const bool live = c < batch;
    for (int k = threadIdx.x; k < Kpad; k += blockDim.x) {
        double fx = 0.0, bv = 0.0;
        if (!live) {
        } else if (k == 0) {
            fx = 1.0;
        } else if (k <= n) {
            if (x) fx = x[(size_t)c * n + k - 1];
            if (v) bv = v[(size_t)c * n + k - 1];
        }
        zf[k] = fx;
        zb[k] = bv;
    }
}

__global__ void k_build_z(int batch, int n, int Kpad, const double* __restrict__ x, const double* __restrict__ v,
                          double* __restrict__ Z, int zrow0) {
    const int c = blockIdx.x;
    if (c >= zrow0) return;
    build_z_row(c, batch, n, Kpad, x, v, Z, zrow0);
}

// The rows of `count` spectrahedra in one launch: zrow0 blocks per instance.
__global__ void k_build_z_multi(const ZRows* __restrict__ d, int batch, int zrow0) {
    const ZRows& z = d[blockIdx.x / zrow0];
    build_z_row(blockIdx.x % zrow0, batch, z.n, z.Kpad, z.x, z.v, z.Z, zrow0);
}

// Compact rows: for j < count, rows k * zc0 + j of Zc = rows k * z0 + list[j]
// of Z (k < nrows); rows count <= j < zc0 of Zc are zero.
__global__ void k_gather_rows(int count, int zc0, int nrows, int Kpad, const int32_t* __restrict__ list,
                              const double* __restrict__ Z, int z0, double* __restrict__ Zc) {
    const int j = blockIdx.x;
    if (j >= zc0) return;
    const int c = j < count ? list[j] : -1;
    for (int k = 0; k < nrows; ++k) {
        double* dst = Zc + ((size_t)k * zc0 + j) * Kpad;
        const double* src = c >= 0 ? Z + ((size_t)k * z0 + c) * Kpad : nullptr;
        for (int i = threadIdx.x; i < Kpad; i += blockDim.x) dst[i] = src ? src[i] : 0.0;
    }
}

hipError_t launch_gather_rows(int count, int zc0, int nrows, int Kpad, const int32_t* list, const double* Z, int z0,
                              double* Zc, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (zc0 < count) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather_rows, dim3(zc0), dim3(64), 0, s, count, zc0, nrows, Kpad, list, Z, z0, Zc);
    return hipGetLastError();
}

hipError_t launch_build_z(int batch, int n, int Kpad, const double* x, const double* v, double* Z, int zrow0,
                          hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    if (zrow0 < batch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_build_z, dim3(zrow0), dim3(64), 0, s, batch, n, Kpad, x, v, Z, zrow0);
    return hipGetLastError();
}

hipError_t launch_build_z_multi(const ZRows* d, int count, int batch, int zrow0, hipStream_t s) {
    if (batch <= 0 || count <= 0) return hipSuccess;
    if (zrow0 < batch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_build_z_multi, dim3(count * zrow0), dim3(64), 0, s, d, batch, zrow0);
    return hipGetLastError();
}

// Rows k * zrow0 + c (k < nrows) of Z from the coefficient rows
// coef[c][k][0..n] of curve c, zero-padded to Kpad.
__global__ void k_build_z_coef(int batch, int n, int Kpad, int nrows, const double* __restrict__ coef,
                               double* __restrict__ Z, int zrow0) {
    const int c = blockIdx.x;
    if (c >= batch) return;
    for (int k = 0; k < 3; ++k) {
        double* z = Z + ((size_t)k * zrow0 + c) * Kpad;
        for (int i = threadIdx.x; i < Kpad; i += blockDim.x)
            z[i] = (k < nrows && i <= n) ? coef[((size_t)c * nrows + k) * (n + 1) + i] : 0.0;
    }
}

// All `nrows` coefficient rows of a curve: row k of curve c at k zrow0 + c.
__global__ void k_build_z_rows(int batch, int n, int Kpad, int nrows, const double* __restrict__ coef,
                               double* __restrict__ Z, int zrow0) {
    const int c = blockIdx.x;
    if (c >= batch) return;
    for (int k = 0; k < nrows; ++k) {
        double* z = Z + ((size_t)k * zrow0 + c) * Kpad;
        for (int i = threadIdx.x; i < Kpad; i += blockDim.x)
            z[i] = i <= n ? coef[((size_t)c * nrows + k) * (n + 1) + i] : 0.0;
    }
}

hipError_t launch_build_z_rows(int batch, int n, int Kpad, int nrows, const double* coef, double* Z, int zrow0,
                               hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_z_rows, dim3(batch), dim3(64), 0, s, batch, n, Kpad, nrows, coef, Z, zrow0);
    return hipGetLastError();
}

hipError_t launch_build_z_coef(int batch, int n, int Kpad, int nrows, const double* coef, double* Z, int zrow0,
                               hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_build_z_coef, dim3(batch), dim3(64), 0, s, batch, n, Kpad, nrows, coef, Z, zrow0);
    return hipGetLastError();
}

// Reflection (Alg. REFLECTION): w from the normal GEMM (dense hit, Lemma
// "Gradient of det F") or the hit row's coefficients (diagonal hit), oriented
// outward, and s = v - 2 <v, w_hat> w_hat.  One wave per chain.
__global__ __launch_bounds__(256) void k_reflect_finish(ReflectArgs a) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (c >= a.batch) return;
    const int n = a.n;
    const double* v = a.v + (size_t)c * n;
    double* s = a.s_out + (size_t)c * n;
    double* w = a.w_out ? a.w_out + (size_t)c * n : nullptr;
    int32_t st = a.status[c];
    const int hit = a.hit[c];
    const double tp = a.tp[c];
    if (st == SPEC_NOT_INTERIOR) {
        for (int i = lane; i < n; i += 64) {
            s[i] = NAN;
            if (w) w[i] = NAN;
        }
        return;
    }
    if (hit == HIT_NONE || !isfinite(tp)) {
        for (int i = lane; i < n; i += 64) {
            s[i] = v[i];
            if (w) w[i] = 0.0;
        }
        return;
    }
    // gather the raw normal
    double nn = 0.0, vw = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double wi = hit == HIT_DENSE ? a.wn[(size_t)c * a.ldwn + i]
                                           : a.Astk[(size_t)(i + 1) * a.ldA + a.P + hit];
        nn += wi * wi;
        vw += wi * v[i];
    }
    nn = wave_sum(nn);
    vw = wave_sum(vw);
    if (!(nn > 0.0)) {
        for (int i = lane; i < n; i += 64) {
            s[i] = v[i];
            if (w) w[i] = 0.0;
        }
        if (lane == 0 && st == SPEC_OK) a.status[c] = SPEC_NONSMOOTH;
        return;
    }
    // two pieces of the boundary meet at the hit: the normal of the one that
    // was found is used, and the status says so
    if (a.flags && (a.flags[c] & SPEC_FLAG_TIE) && lane == 0 && st == SPEC_OK) a.status[c] = SPEC_NONSMOOTH;
    const double inv = 1.0 / sqrt(nn);
    const double sgn = vw < 0.0 ? -1.0 : 1.0;
    const double dvw = fabs(vw) * inv;  // <v, w_hat> with w_hat outward
    for (int i = lane; i < n; i += 64) {
        const double wi = hit == HIT_DENSE ? a.wn[(size_t)c * a.ldwn + i]
                                           : a.Astk[(size_t)(i + 1) * a.ldA + a.P + hit];
        const double wh = sgn * wi * inv;
        s[i] = v[i] - 2.0 * dvw * wh;
        if (w) w[i] = wh;
    }
}

hipError_t launch_reflect_finish(const ReflectArgs& a, hipStream_t s) {
    if (a.batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reflect_finish, dim3((a.batch + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace spec

namespace spec {

__global__ void k_status_to_flag(int batch, const int32_t* __restrict__ st, int8_t* __restrict__ flag) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < batch) flag[c] = st[c] == SPEC_OK ? 1 : 0;
}

hipError_t launch_status_to_flag(int batch, const int32_t* st, int8_t* flag, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_status_to_flag, dim3((batch + 255) / 256), dim3(256), 0, s, batch, st, flag);
    return hipGetLastError();
}

}  // namespace spec

namespace spec {

// out[0] = sum_r M[r * ld + col] over r < rows (one block, deterministic order).
__global__ void k_sum_col(int rows, const double* __restrict__ M, int ld, int col, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) s += M[(size_t)r * ld + col];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_sum_col(int rows, const double* M, int ld, int col, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_col, dim3(1), dim3(256), 0, s, rows, M, ld, col, out);
    return hipGetLastError();
}

}  // namespace spec
