// Device helpers shared by the kernel sources: wave and block reductions,
// the canonical FP32 residual, compensated residuals of FP64 planes, the
// Philox4x64-10 generator and the FP32 three-point plane.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ppk {

// v plus the value of the lane that DPP control CTRL selects (0 in rows that
// ROW_MASK leaves out).
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int dpp_add(int v) {
    return v + __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, false);
}

// Sum over the wave, returned to every lane: quad permutes and row rotations
// give each row's sum, the row broadcasts carry it into lane 63 (DPP, no LDS).
__device__ __forceinline__ int wave_sum(int v) {
    v = dpp_add<0xB1>(v);        // quad_perm [1,0,3,2]
    v = dpp_add<0x4E>(v);        // quad_perm [2,3,0,1]
    v = dpp_add<0x124>(v);       // row_ror:4
    v = dpp_add<0x128>(v);       // row_ror:8
    v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long w = __shfl_xor(v, o);
        v = v > w ? v : w;
    }
    return v;
}

// Max (or min) over the wave, returned to every lane, by the same DPP steps.
template <bool MAX, int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int dpp_ext(int v) {
    // all rows enabled: every source lane is valid, so no old value is needed
    // and the compiler can fold the permute into the min / max
    const int b = ROW_MASK == 0xF ? __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true)
                                  : __builtin_amdgcn_update_dpp(v, v, CTRL, ROW_MASK, 0xF, false);
    return MAX ? max(v, b) : min(v, b);
}

template <bool MAX>
__device__ __forceinline__ int wave_ext(int v) {
    v = dpp_ext<MAX, 0xB1>(v);
    v = dpp_ext<MAX, 0x4E>(v);
    v = dpp_ext<MAX, 0x124>(v);
    v = dpp_ext<MAX, 0x128>(v);
    v = dpp_ext<MAX, 0x142, 0xA>(v);
    v = dpp_ext<MAX, 0x143, 0xC>(v);
    return __builtin_amdgcn_readlane(v, 63);
}

// Sum over the 256 threads of a block; every thread gets the total.
__device__ __forceinline__ int block_sum(int v, int* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// Two block sums at once (sh holds 8 ints).
__device__ __forceinline__ void block_sum2(int& a, int& b, int* sh) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) {
        sh[w] = a;
        sh[4 + w] = b;
    }
    __syncthreads();
    a = sh[0] + sh[1] + sh[2] + sh[3];
    b = sh[4] + sh[5] + sh[6] + sh[7];
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const unsigned l = threadIdx.x & 63;
    return l ? (~0ull >> (64 - l)) : 0ull;
}

// Stable compaction step for 256 candidates (one per thread): returns this
// thread's rank among the flagged threads before it; *total gets the count.
__device__ __forceinline__ int block_rank(bool flag, int* sh, int* total) {
    const unsigned long long m = __ballot(flag);
    const int w = threadIdx.x >> 6;
    const int in_wave = __popcll(m & lanemask_lt());
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = __popcll(m);
    __syncthreads();
    int before = 0;
    for (int i = 0; i < w; ++i) before += sh[i];
    *total = sh[0] + sh[1] + sh[2] + sh[3];
    return before + in_wave;
}

// block_rank for S steps at once, ordered step-major (all of step 0, then
// step 1, ...), each step by wave then lane; one barrier pair.  sh holds 4 S ints.
template <int S>
__device__ __forceinline__ void block_rank_steps(const bool (&flag)[S], int* sh, int (&rank)[S], int& total) {
    const int w = threadIdx.x >> 6;
    unsigned long long m[S];
#pragma unroll
    for (int k = 0; k < S; ++k) m[k] = __ballot(flag[k]);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < S; ++k) sh[4 * k + w] = __popcll(m[k]);
    __syncthreads();
    int base = 0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        int before = base;
        for (int i = 0; i < 4; ++i) {
            const int n = sh[4 * k + i];
            before += i < w ? n : 0;
            base += n;
        }
        rank[k] = before + __popcll(m[k] & lanemask_lt());
    }
    total = base;
}

// The canonical FP32 residual n.p + d of a hypothesis plane.  Every scorer
// and the refit decide |r| < t with exactly this expression.
__device__ __forceinline__ float canon_res(const float4 h, float x, float y, float z) {
    return fmaf(h.x, x, fmaf(h.y, y, fmaf(h.z, z, h.w)));
}

// Refit planes are FP64; their inlier test evaluates n.p + d for FP32 points
// in compensated FP32 (hi/lo split plane, error-free products, two-sum), which
// is accurate to ~2^-44 of the largest term.
struct SplitPlane {
    float hx, hy, hz, hd, lx, ly, lz, ld;
};

__device__ __forceinline__ SplitPlane split_plane(const double* p) {
    SplitPlane s;
    s.hx = (float)p[0]; s.lx = (float)(p[0] - (double)s.hx);
    s.hy = (float)p[1]; s.ly = (float)(p[1] - (double)s.hy);
    s.hz = (float)p[2]; s.lz = (float)(p[2] - (double)s.hz);
    s.hd = (float)p[3]; s.ld = (float)(p[3] - (double)s.hd);
    return s;
}

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ float refit_res(const SplitPlane& q, float x, float y, float z) {
    const float p0 = q.hx * x, e0 = fmaf(q.hx, x, -p0);
    const float p1 = q.hy * y, e1 = fmaf(q.hy, y, -p1);
    const float p2 = q.hz * z, e2 = fmaf(q.hz, z, -p2);
    float s, t0, t1, t2;
    two_sum(q.hd, p0, s, t0);
    two_sum(s, p1, s, t1);
    two_sum(s, p2, s, t2);
    const float small = ((q.ld + (e0 + e1 + e2)) + (t0 + t1 + t2)) + (q.lx * x + q.ly * y + q.lz * z);
    return s + small;
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies with the published constants, key bumped by the
// published Weyl increments between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t a = hi1 ^ c[1] ^ k0, b = hi0 ^ c[3] ^ k1;
        c[0] = a;
        c[1] = lo1;
        c[2] = b;
        c[3] = lo0;
    }
}

// FP32 plane through three points (the plane model of Alg. 2): n = e1 x e2
// normalised, d = -n.p0, camera-facing (d >= 0); degenerate when
// |e1 x e2| <= 1e-3 |e1||e2|, returned as d = NaN (never an inlier).
__device__ __forceinline__ float4 plane_from_points(float3 p0, float3 p1, float3 p2) {
    const float e1x = p1.x - p0.x, e1y = p1.y - p0.y, e1z = p1.z - p0.z;
    const float e2x = p2.x - p0.x, e2y = p2.y - p0.y, e2z = p2.z - p0.z;
    const float mx = e1y * e2z - e1z * e2y;
    const float my = e1z * e2x - e1x * e2z;
    const float mz = e1x * e2y - e1y * e2x;
    const float mn = sqrtf(mx * mx + my * my + mz * mz);
    const float l1 = sqrtf(e1x * e1x + e1y * e1y + e1z * e1z);
    const float l2 = sqrtf(e2x * e2x + e2y * e2y + e2z * e2z);
    if (!(mn > 1e-3f * l1 * l2)) return make_float4(0.f, 0.f, 0.f, __int_as_float(0x7fc00000));
    float nx = mx / mn, ny = my / mn, nz = mz / mn;
    float d = -(nx * p0.x + ny * p0.y + nz * p0.z);
    if (d < 0.f) {
        nx = -nx; ny = -ny; nz = -nz; d = -d;
    }
    return make_float4(nx, ny, nz, d);
}

}  // namespace ppk
