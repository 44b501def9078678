// Device-side helpers shared by the HIP kernels of the boundary oracle.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spec {

// Packed storage of a symmetric / lower-triangular m x m matrix: row r keeps
// columns 0..r at offset r(r+1)/2.
__host__ __device__ inline int pk(int r, int c) { return (r * (r + 1)) / 2 + c; }

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
// ten rounds of the two 32x32->64 multiplications with the key bumped by the
// golden-ratio and sqrt(3)-1 Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct u4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u4 philox10(u4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        u4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Stream tags (low byte of the fourth counter word).
enum : uint32_t {
    TAG_DIR = 1, TAG_LEN = 2, TAG_POS = 3, TAG_COORD = 4, TAG_MOM = 5, TAG_GAUSS0 = 6, TAG_BALL = 7, TAG_BALL_R = 8,
    TAG_MLP_BATCH = 0x40, TAG_MLP_INIT = 0x41
};

// Two doubles in (0,1), 53 random bits each, from one Philox block.
__device__ __forceinline__ void u01x2(u4 w, double& a, double& b) {
    const double s = 1.0 / 9007199254740992.0;  // 2^-53
    a = ((double)(w.x >> 5) * 67108864.0 + (double)(w.y >> 6) + 0.5) * s;
    b = ((double)(w.z >> 5) * 67108864.0 + (double)(w.w >> 6) + 0.5) * s;
}

__device__ __forceinline__ void draw_u2(uint64_t seed, uint32_t chain, uint32_t step, uint32_t draw,
                                        uint32_t tag, double& a, double& b) {
    u4 c{chain, step, draw, tag};
    u01x2(philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32)), a, b);
}

// Normals 2d and 2d+1 of a stream by Box-Muller.
__device__ __forceinline__ void normal_pair(uint64_t seed, uint32_t chain, uint32_t step, uint32_t d,
                                            uint32_t tag, double& g0, double& g1) {
    double a, b;
    draw_u2(seed, chain, step, d, tag, a, b);
    const double r = sqrt(-2.0 * log(a));
    double sn, cs;
    sincospi(2.0 * b, &sn, &cs);
    g0 = r * cs;
    g1 = r * sn;
}

// ---------------------------------------------------------------------------
// Reductions over a workgroup (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// A value the whole wave agrees on, moved to scalar registers.
__device__ __forceinline__ double wave_uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Workgroup barrier that orders LDS only: global stores in flight are not
// waited for (they are not read back by other threads before a full fence).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum over the block with LDS-only barriers (see block_sum).
__device__ inline double block_sum_lds(double v, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    lds_barrier();
    if (lane == 0) red[wid] = v;
    lds_barrier();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

// Sum over the block; `red` is LDS scratch of at least blockDim/64 doubles.
// Contains barriers: every thread of the block must call it.
__device__ inline double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

}  // namespace spec
