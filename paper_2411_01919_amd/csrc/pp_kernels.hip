// HIP kernels of the plane-extraction path for gfx950 (MI355X, wave64).
//
// Stage map (arXiv 2411.01919):
//   k_diffuse_wc     Perona-Malik diffusion, Eq. 1 / Alg. 1: T iterations fused
//                    per pass, FP32 on delta = I - I0, the iterate in registers
//                    (one wave per column strip); k_diffuse: the same on LDS tiles
//   k_normals        back-projection (Alg. 2) + Sobel normal image (Eq. 2);
//                    in batches also the valid-list chunk counts
//   k_valid_*        row-major list of depth-valid pixels (Alg. 2 point set)
//   k_list0          the round-0 scoring list: every position of the image's
//                    8x8-block scan (NaN for no point) with the bounding boxes
//                    of its 64-point tiles
//   k_round_start    3-point hypotheses from Philox4x64-10 (Alg. 2)
//   k_score_tiles    inlier counts, point-to-plane distance < t (Eq. 3, Alg. 2):
//                    tiles decided from their boxes, the rest point by point
//                    on the vector ALUs or the matrix cores (k_score: every
//                    point)
//   k_refit_*        selection of j*, FP64 moments of its inliers, the
//                    least-squares plane (solved in every block of the final
//                    pass) and its inliers per chunk
//   k_apply          remove / label the refit plane's inliers; the next
//                    round's list with the boxes of its tiles
//
// Every kernel takes a device table of FrameDev and reads its frame from
// blockIdx.z (k_round_start: from a 1-D grid, XCD-aware for the hypotheses),
// so one launch serves one frame or a ragged batch alike.

#include <math.h>

#include "pp_device.h"
#include "pp_internal.h"

namespace ppk {

// Read-only pointers in the global address space: their loads need not wait
// for earlier LDS or generic stores, which a generic (flat) load might alias.
typedef const __attribute__((address_space(1))) uint8_t* gu8_cptr;
typedef const __attribute__((address_space(1))) int32_t* gi32_cptr;
typedef const __attribute__((address_space(1))) float* gf32_cptr;
typedef const __attribute__((address_space(1))) double* gf64_cptr;

__device__ __forceinline__ float3 load_point(const FrameDev& f, int off) {
    const size_t plane = (size_t)f.H * f.pitch;
    return make_float3(f.pts[off], f.pts[plane + off], f.pts[2 * plane + off]);
}

__device__ __forceinline__ bool hyp_valid(const float4 h) { return h.w == h.w; }

// Round r's flags by one scalar load.  No kernel writes the record it reads
// this way (each round's record is written by the kernels before it).
__device__ __forceinline__ RoundRec round_rec(const FrameDev& f, int r) {
    typedef int v8i_t __attribute__((ext_vector_type(8)));
    typedef const __attribute__((address_space(4))) v8i_t* ci8_ptr;
    const v8i_t v = ((ci8_ptr)(f.st->round + r))[0];
    return RoundRec{v[0], v[1], v[2], v[3], v[4], {v[5], v[6], v[7]}};
}

// exp(-(x/kappa)^2) as 2^-a with the hardware exponential (v_exp_f32, about
// 1 ulp).  It skips the library's rescaling for subnormal results: those would
// contribute less than 1e-30 mm to a flux.
__device__ __forceinline__ float g_exp(float a) { return __builtin_amdgcn_exp2f(-a); }

// ------------------------------------------------------------------ diffusion
// One pass = `it` (<= T) explicit iterations on a TX x TY tile whose LDS copy
// carries a T-pixel halo.  Iteration k updates the tile grown by T - k (for
// it == T) pixels, so the last one is exact on the tile.  The iterate is kept
// as delta = I - I0 with I0 the integer input, so the integer part of every
// edge difference, (I0_q - I0_p), is exact and loop-invariant (precomputed).
// Each iteration, every pixel computes the fluxes g(D) D of its four edges
// from the previous iterate and writes its new value to the other LDS buffer
// (one barrier per iteration).
template <int TX, int TY, int T>
__global__ __launch_bounds__(kBlock) void k_diffuse(const FrameDev* __restrict__ tab, int it, int first, int last,
                                                     int src, int dst) {
    const FrameDev& f = tab[blockIdx.z];
    const int W = f.W, H = f.H;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    if (x0 >= W || y0 >= H) return;
    constexpr int EW = TX + 2 * T, EH = TY + 2 * T, EN = EW * EH;
    constexpr int NPT = (EN + kBlock - 1) / kBlock;  // extended pixels per thread
    __shared__ float s_i0[EN];
    __shared__ float s_d[2][EN];  // the iterate, read from one while the other is written
    const float* __restrict__ din = f.delta[src];
    for (int e = threadIdx.x; e < EN; e += kBlock) {
        const int ex = e % EW, ey = e / EW;
        const int x = x0 - T + ex, y = y0 - T + ey;
        float i0 = 0.f, d = 0.f;
        if (x >= 0 && x < W && y >= 0 && y < H) {
            i0 = (float)f.depth[(size_t)y * f.pitch + x];
            if (!first && i0 > 0.f) d = din[(size_t)y * W + x];
        }
        s_i0[e] = i0;
        s_d[0][e] = d;
    }
    __syncthreads();
    // loop-invariant data of this thread's pixels: the integer part of the
    // east and south differences, and which of the four edges are open
    float i0p[NPT], dIe[NPT], dIs[NPT];
    uint32_t open[NPT];  // bit 0 pixel valid, 1 east, 2 south, 3 west, 4 north
    int exy[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const int e = threadIdx.x + q * kBlock;
        const int ex = e % EW, ey = e / EW;
        exy[q] = (ex << 16) | ey;
        open[q] = 0u; dIe[q] = 0.f; dIs[q] = 0.f; i0p[q] = 0.f;
        if (e < EN) {
            const float i0 = s_i0[e];
            i0p[q] = i0;
            if (i0 > 0.f) {
                uint32_t o = 1u;
                if (ex + 1 < EW) { const float q0 = s_i0[e + 1]; o |= q0 > 0.f ? 2u : 0u; dIe[q] = q0 - i0; }
                if (ey + 1 < EH) { const float q0 = s_i0[e + EW]; o |= q0 > 0.f ? 4u : 0u; dIs[q] = q0 - i0; }
                if (ex >= 1 && s_i0[e - 1] > 0.f) o |= 8u;
                if (ey >= 1 && s_i0[e - EW] > 0.f) o |= 16u;
                open[q] = o;
            }
        }
    }
    const float lam = f.lambda, gs = f.g_scale;
    const bool rational = f.edge_stop == PP_EDGE_RATIONAL;
    auto flux = [&](float D) {
        const float a = D * D * gs;
        return (rational ? 1.0f / (1.0f + a) : g_exp(a)) * D;
    };
    int cur = 0;
    for (int k = 1; k <= it; ++k) {
        const int s = T - it + k;  // pixels updated this iteration: [s, EW - s) x [s, EH - s)
        const float* __restrict__ sd = s_d[cur];
        float* __restrict__ nd = s_d[cur ^ 1];
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const int e = threadIdx.x + q * kBlock;
            const int ex = exy[q] >> 16, ey = exy[q] & 0xFFFF;
            if (!(open[q] & 1u) || ex < s || ex >= EW - s || ey < s || ey >= EH - s) continue;
            const uint32_t o = open[q];
            const float dp = sd[e];
            // each edge's flux g(D) D with D = I_q - I_p taken in the same operand order by
            // both of its pixels (delta form: the integer part is exact), so it leaves one
            // pixel exactly as it enters the other; closed edges (holes, border) carry none
            const float fe = (o & 2u) ? flux(dIe[q] + (sd[e + 1] - dp)) : 0.f;
            const float fs = (o & 4u) ? flux(dIs[q] + (sd[e + EW] - dp)) : 0.f;
            const float fw = (o & 8u) ? flux((i0p[q] - s_i0[e - 1]) + (dp - sd[e - 1])) : 0.f;
            const float fn = (o & 16u) ? flux((i0p[q] - s_i0[e - EW]) + (dp - sd[e - EW])) : 0.f;
            nd[e] = dp + lam * ((fe - fw) + (fs - fn));
        }
        __syncthreads();
        cur ^= 1;
    }
    float* __restrict__ dout = f.delta[dst];
    for (int e = threadIdx.x; e < TX * TY; e += kBlock) {
        const int tx = e % TX, ty = e / TX;
        const int x = x0 + tx, y = y0 + ty;
        if (x >= W || y >= H) continue;
        const int ee = (ty + T) * EW + (tx + T);
        const float i0 = s_i0[ee];
        const float d = i0 > 0.f ? s_d[cur][ee] : 0.f;
        if (last)
            f.dmm[(size_t)y * f.pitch + x] = i0 > 0.f ? i0 + d : 0.f;
        else
            dout[(size_t)y * W + x] = d;
    }
}

// Lane l receives lane l - 1's value (DPP wave_shr:1); lane 0 receives 0.
__device__ __forceinline__ float from_west_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
// Lane l receives lane l + 1's value (DPP wave_shl:1); lane 63 receives 0.
__device__ __forceinline__ float from_east_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}

// The same iteration as k_diffuse with the iterate held in registers: lane l
// of a wave owns image column x0 - T + l and the R = TY + 2T rows around the
// wave's TY output rows.  A pixel's east neighbour is the next lane (a DPP
// shift), its south neighbour the next register, so each edge's flux g(D) D is
// computed once per iteration, by the pixel west (north) of it, and reaches
// the other pixel by a lane shift (the previous row's value); no LDS and no
// barriers.  After k iterations lanes [k, 63 - k] and rows [k, R - 1 - k] hold
// exact values, so a wave writes its 64 - 2T middle columns.  Every flux is
// the expression k_diffuse evaluates for that edge, so the results are
// bitwise the same.
template <int TY, int T, bool RATIONAL>
__device__ __forceinline__ void diffuse_wc_body(const FrameDev& f, int it, int first, int last, int src, int dst) {
    constexpr int R = TY + 2 * T;
    constexpr int OW = 64 - 2 * T;  // output columns per wave
    const int W = f.W, H = f.H;
    const int lane = threadIdx.x & 63;
    const int ox0 = (blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * OW;
    const int y0 = blockIdx.y * TY;
    if (ox0 >= W || y0 >= H) return;  // whole waves only: nothing below synchronises across waves
    const int x = ox0 - T + lane;
    const bool xin = x >= 0 && x < W;
    const int xc = min(max(x, 0), W - 1);
    typedef const __attribute__((address_space(1))) uint16_t* gu16_ptr;
    typedef const __attribute__((address_space(1))) float* gf32_ptr;
    const gu16_ptr dep = (gu16_ptr)f.depth;
    const gf32_ptr din = (gf32_ptr)f.delta[src];
    float d[R], dIe[R], dIs[R], ce[R], cs[R];
    {
        // every row's loads issued at once: addresses clamped into the frame, values masked after
        float i0[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = y0 - T + r;
            const int yc = min(max(y, 0), H - 1);
            const float v = (float)dep[(size_t)yc * f.pitch + xc];
            i0[r] = (xin && y >= 0 && y < H) ? v : 0.f;
        }
        if (first) {
#pragma unroll
            for (int r = 0; r < R; ++r) d[r] = 0.f;
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int yc = min(max(y0 - T + r, 0), H - 1);
                const float v = din[(size_t)yc * W + xc];
                d[r] = i0[r] > 0.f ? v : 0.f;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float ie = from_east_lane(i0[r]);  // 0 beyond the wave: a closed edge in the halo
            dIe[r] = ie - i0[r];
            ce[r] = (i0[r] > 0.f && ie > 0.f) ? 1.f : 0.f;
            if (r + 1 < R) {
                dIs[r] = i0[r + 1] - i0[r];
                cs[r] = (i0[r] > 0.f && i0[r + 1] > 0.f) ? 1.f : 0.f;
            } else {
                dIs[r] = 0.f;
                cs[r] = 0.f;
            }
        }
    }
    const float lam = f.lambda, gs = f.g_scale;
    auto flux = [&](float D) {
        const float a = D * D * gs;
        return (RATIONAL ? 1.0f / (1.0f + a) : g_exp(a)) * D;
    };
#pragma unroll
    for (int k = 1; k <= T; ++k) {
        if (k <= T - it) continue;  // a short pass runs its `it` iterations as the last ones of T
        // rows [k, R - 1 - k]; the south flux of row k - 1 is the first north flux
        float fn = flux(dIs[k - 1] + (d[k] - d[k - 1])) * cs[k - 1];
#pragma unroll
        for (int r = k; r <= R - 1 - k; ++r) {
            const float dp = d[r];
            const float fe = flux(dIe[r] + (from_east_lane(dp) - dp)) * ce[r];
            const float fs = flux(dIs[r] + (d[r + 1] - dp)) * cs[r];
            const float fw = from_west_lane(fe);
            d[r] = dp + lam * ((fe - fw) + (fs - fn));
            fn = fs;
        }
    }
    if (lane < T || lane >= 64 - T || x >= W) return;
    float* __restrict__ dout = f.delta[dst];
#pragma unroll
    for (int r = T; r < T + TY; ++r) {
        const int y = y0 - T + r;
        if (y >= H) break;
        if (last) {
            const float i0 = (float)f.depth[(size_t)y * f.pitch + x];
            f.dmm[(size_t)y * f.pitch + x] = i0 > 0.f ? i0 + d[r] : 0.f;
        } else {
            dout[(size_t)y * W + x] = d[r];
        }
    }
}

template <int TY, int T>
__global__ __launch_bounds__(kBlock) void k_diffuse_wc(const FrameDev* __restrict__ tab, int it, int first, int last,
                                                        int src, int dst) {
    const FrameDev& f = tab[blockIdx.z];
    if (f.edge_stop == PP_EDGE_RATIONAL)
        diffuse_wc_body<TY, T, true>(f, it, first, last, src, dst);
    else
        diffuse_wc_body<TY, T, false>(f, it, first, last, src, dst);
}

// Other discretisations of Eq. 1, on the same tiling, temporal blocking and
// delta form as k_diffuse (fixed 64 x 16 tiles, up to kVarT iterations a pass):
//  PP_DIFFUSE_PIXEL  Alg. 1 as printed.  Each pixel takes c_p = g(|grad I_p|),
//                    the gradient from central differences, or a one-sided
//                    difference when only one neighbour along that axis is
//                    valid (0 with none), and adds lam c_p times the sum of
//                    (I_q - I_p) over its valid 4-neighbours.  A pixel's update
//                    is computed from the old image first (s_u), then applied.
//  PP_DIFFUSE_EDGE8  per-edge fluxes over the 8-neighbourhood.  Each pixel owns
//                    its E, S, SE and SW edge; a diagonal flux is
//                    1/2 g(|D| / sqrt 2) D.  Every flux is computed once and
//                    enters both of its pixels with opposite signs.
constexpr int kVarTX = 64, kVarTY = 16, kVarT = 5;

__device__ __forceinline__ float edge_g(float a, bool rational) { return rational ? 1.0f / (1.0f + a) : g_exp(a); }

template <int SCHEME>
__global__ __launch_bounds__(kBlock) void k_diffuse_var(const FrameDev* __restrict__ tab, int it, int first, int last,
                                                        int src, int dst) {
    constexpr int TX = kVarTX, TY = kVarTY, T = kVarT;
    constexpr int EW = TX + 2 * T, EH = TY + 2 * T, EN = EW * EH;
    constexpr int NA = SCHEME == PP_DIFFUSE_EDGE8 ? 4 : 1;  // per-pixel work arrays
    const FrameDev& f = tab[blockIdx.z];
    const int W = f.W, H = f.H;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    if (x0 >= W || y0 >= H) return;
    __shared__ float s_i0[EN];
    __shared__ float s_d[EN];
    __shared__ float s_a[NA][EN];  // PIXEL: the update; EDGE8: E, S, SE, SW fluxes
    const float* __restrict__ din = f.delta[src];
    for (int e = threadIdx.x; e < EN; e += kBlock) {
        const int x = x0 - T + e % EW, y = y0 - T + e / EW;
        float i0 = 0.f, d = 0.f;
        if (x >= 0 && x < W && y >= 0 && y < H) {
            i0 = (float)f.depth[(size_t)y * f.pitch + x];
            if (!first && i0 > 0.f) d = din[(size_t)y * W + x];
        }
        s_i0[e] = i0;
        s_d[e] = d;
    }
    __syncthreads();
    const float lam = f.lambda, gs = f.g_scale;
    const bool rational = f.edge_stop == PP_EDGE_RATIONAL;
    for (int k = 1; k <= it; ++k) {
        const int s = T - it + k;  // pixels updated this iteration: [s, EW - s) x [s, EH - s)
        for (int e = threadIdx.x; e < EN; e += kBlock) {
            const int ex = e % EW, ey = e / EW;
            if (SCHEME == PP_DIFFUSE_PIXEL) {
                if (ex < s || ex >= EW - s || ey < s || ey >= EH - s) continue;
                const float i0 = s_i0[e];
                if (!(i0 > 0.f)) continue;
                const float dp = s_d[e];
                // differences I_q - I_p of the four neighbours (integer part exact)
                const bool ve = s_i0[e + 1] > 0.f, vw = s_i0[e - 1] > 0.f;
                const bool vs = s_i0[e + EW] > 0.f, vn = s_i0[e - EW] > 0.f;
                const float De = ve ? (s_i0[e + 1] - i0) + (s_d[e + 1] - dp) : 0.f;
                const float Dw = vw ? (s_i0[e - 1] - i0) + (s_d[e - 1] - dp) : 0.f;
                const float Ds = vs ? (s_i0[e + EW] - i0) + (s_d[e + EW] - dp) : 0.f;
                const float Dn = vn ? (s_i0[e - EW] - i0) + (s_d[e - EW] - dp) : 0.f;
                const float gx = ve && vw ? 0.5f * ((s_i0[e + 1] - s_i0[e - 1]) + (s_d[e + 1] - s_d[e - 1]))
                                          : (De - Dw);
                const float gy = vs && vn ? 0.5f * ((s_i0[e + EW] - s_i0[e - EW]) + (s_d[e + EW] - s_d[e - EW]))
                                          : (Ds - Dn);
                const float c = edge_g((gx * gx + gy * gy) * gs, rational);
                s_a[0][e] = lam * c * ((De + Dw) + (Ds + Dn));
            } else {
                // fluxes of edges whose both pixels hold this iteration's input: [s-1, EW-s+1)^2
                if (ex < s - 1 || ex >= EW - s + 1 || ey < s - 1 || ey >= EH - s + 1) continue;
                const float i0 = s_i0[e], dp = s_d[e];
                const bool vp = i0 > 0.f;
                float fE = 0.f, fS = 0.f, fSE = 0.f, fSW = 0.f;
                if (vp && ex < EW - s && s_i0[e + 1] > 0.f) {
                    const float D = (s_i0[e + 1] - i0) + (s_d[e + 1] - dp);
                    fE = edge_g(D * D * gs, rational) * D;
                }
                if (vp && ey < EH - s) {
                    if (s_i0[e + EW] > 0.f) {
                        const float D = (s_i0[e + EW] - i0) + (s_d[e + EW] - dp);
                        fS = edge_g(D * D * gs, rational) * D;
                    }
                    if (ex < EW - s && s_i0[e + EW + 1] > 0.f) {
                        const float D = (s_i0[e + EW + 1] - i0) + (s_d[e + EW + 1] - dp);
                        fSE = 0.5f * edge_g(0.5f * D * D * gs, rational) * D;
                    }
                    if (ex >= s && s_i0[e + EW - 1] > 0.f) {
                        const float D = (s_i0[e + EW - 1] - i0) + (s_d[e + EW - 1] - dp);
                        fSW = 0.5f * edge_g(0.5f * D * D * gs, rational) * D;
                    }
                }
                s_a[0][e] = fE;
                s_a[NA > 1 ? 1 : 0][e] = fS;
                s_a[NA > 2 ? 2 : 0][e] = fSE;
                s_a[NA > 3 ? 3 : 0][e] = fSW;
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < EN; e += kBlock) {
            const int ex = e % EW, ey = e / EW;
            if (ex < s || ex >= EW - s || ey < s || ey >= EH - s || !(s_i0[e] > 0.f)) continue;
            if (SCHEME == PP_DIFFUSE_PIXEL) {
                s_d[e] += s_a[0][e];
            } else {
                const float sum = (s_a[0][e] - s_a[0][e - 1]) + (s_a[NA > 1 ? 1 : 0][e] - s_a[NA > 1 ? 1 : 0][e - EW]) +
                                  ((s_a[NA > 2 ? 2 : 0][e] - s_a[NA > 2 ? 2 : 0][e - EW - 1]) +
                                   (s_a[NA > 3 ? 3 : 0][e] - s_a[NA > 3 ? 3 : 0][e - EW + 1]));
                s_d[e] += lam * sum;
            }
        }
        __syncthreads();
    }
    float* __restrict__ dout = f.delta[dst];
    for (int e = threadIdx.x; e < TX * TY; e += kBlock) {
        const int tx = e % TX, ty = e / TX;
        const int x = x0 + tx, y = y0 + ty;
        if (x >= W || y >= H) continue;
        const int ee = (ty + T) * EW + (tx + T);
        const float i0 = s_i0[ee];
        const float d = i0 > 0.f ? s_d[ee] : 0.f;
        if (last)
            f.dmm[(size_t)y * f.pitch + x] = i0 > 0.f ? i0 + d : 0.f;
        else
            dout[(size_t)y * W + x] = d;
    }
}

// Zero iterations: the diffused image is the input.
__global__ __launch_bounds__(kBlock) void k_diffuse_copy(const FrameDev* __restrict__ tab) {
    const FrameDev& f = tab[blockIdx.z];
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= f.W || y >= f.H) return;
    const size_t o = (size_t)y * f.pitch + x;
    f.dmm[o] = (float)f.depth[o];
}

// ------------------------------------------------------------------ normals
// Back-projection P = z ((u-cx)/fx, (v-cy)/fy, 1) and the Sobel normal
// n = -(Sx P x Sy P)/|.|.  Because the ray is affine in (u, v) and Sobel
// weights sum to zero, Sx P = z_c (8/fx, 0, 0) + sum_k wx_k (z_k - z_c) ray_k
// (and likewise for Sy): evaluating it in that form avoids the cancellation of
// summing nearly equal points.  Depth is kept in mm (a common scale factor).
// Element i of a row-major plane in the global address space, addressed by a
// 32-bit byte offset from a uniform base (one VGPR offset per access, no 64-bit
// address arithmetic).  Requires i * sizeof(T) < 2^32: a plane holds at most
// 2^30 pixels.
typedef __attribute__((address_space(1))) char gbyte;
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* plane_at(T* base, uint32_t i) {
    return (__attribute__((address_space(1))) T*)((gbyte*)base + (i * (uint32_t)sizeof(T)));
}
__device__ __forceinline__ float plane_ld(const float* base, uint32_t i) {
    return *(const __attribute__((address_space(1))) float*)((const gbyte*)base + i * 4u);
}

// Point and normal of pixel (x, y) from its 3x3 depth window nb (mm; values
// outside the frame are never used): the back-projected point (zero without
// depth), the unit normal of the product-rule Sobel responses (zero unless
// the pixel is interior with a full window and a non-degenerate cross
// product) and the flags (1: depth, 2: normal).
__device__ __forceinline__ uint8_t normal_pixel(const FrameDev& f, int x, int y, const float (&nb)[3][3], float& px,
                                                float& py, float& pz, float& n0, float& n1, float& n2) {
    const float I = nb[1][1];
    const bool dv = I > 0.f;
    px = py = pz = 0.f;
    if (dv) {
        const float z = I / 1000.0f;
        px = z * ((float)x - f.cx) / f.fx;
        py = z * ((float)y - f.cy) / f.fy;
        pz = z;
    }
    bool nv = dv && x >= 1 && x <= f.W - 2 && y >= 1 && y <= f.H - 2;
    n0 = n1 = n2 = 0.f;
    if (nv) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) nv = nv && (nb[j][i] > 0.f);
        if (nv) {
            // sums of w * dI * (u - cx), w * dI * (v - cy), w * dI for both kernels;
            // w dI is exact (w is 0, +-1 or +-2), one rounding per term
            float ax = 0.f, bx = 0.f, cx_ = 0.f, ay = 0.f, by = 0.f, cy_ = 0.f;
            const float wrow[3] = {1.f, 2.f, 1.f};
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const float wx = (float)(i - 1) * wrow[j];  // Sobel x: [-1 0 1] x [1 2 1]^T
                    const float wy = (float)(j - 1) * wrow[i];  // Sobel y: its transpose
                    if (wx == 0.f && wy == 0.f) continue;
                    const float dI = nb[j][i] - I;
                    const float uu = (float)(x + i - 1) - f.cx;
                    const float vv = (float)(y + j - 1) - f.cy;
                    const float ex = wx * dI, ey = wy * dI;
                    ax = fmaf(ex, uu, ax); bx = fmaf(ex, vv, bx); cx_ += ex;
                    ay = fmaf(ey, uu, ay); by = fmaf(ey, vv, by); cy_ += ey;
                }
            // the Sobel responses of the points: the image-plane ones scaled by 1/fx, 1/fy
            const float ifx = f.ifx, ify = f.ify;
            const float sxx = (8.f * I + ax) * ifx, sxy = bx * ify, sxz = cx_;
            const float syx = ay * ifx, syy = (8.f * I + by) * ify, syz = cy_;
            const float mx = sxy * syz - sxz * syy;
            const float my = sxz * syx - sxx * syz;
            const float mz = sxx * syy - sxy * syx;
            const float m2 = fmaf(mx, mx, fmaf(my, my, mz * mz));
            nv = m2 > 0.f;
            if (nv) {
                const float inv = -__frsqrt_rn(m2);
                n0 = mx * inv;
                n1 = my * inv;
                n2 = mz * inv;
            }
        }
    }
    return (uint8_t)((dv ? 1 : 0) | (nv ? 2 : 0));
}

// Points, normals and flags of one 1024-pixel row-major chunk per block, 4
// consecutive pixels per thread.  Four pixels of one row share one 3x6
// window (a 16-byte load per row where rows are 16-byte aligned) and are
// stored 16 bytes per plane.  With count set, the block also writes its
// chunk's number of depth-valid pixels for the valid list (and block 0 resets
// the frame's |p|_1 bound), which makes the separate count pass unnecessary.
__global__ __launch_bounds__(kBlock) void k_normals(const FrameDev* __restrict__ tab, int count) {
    __shared__ int sh[4];
    const FrameDev& f = tab[blockIdx.z];
    const int W = f.W, H = f.H, pitch = f.pitch;
    const int npx = W * H;
    const int c = blockIdx.x;
    if (c * kValidChunk >= npx) return;  // the whole block: this frame has fewer chunks
    if (count && c == 0 && threadIdx.x == 0) f.st->p1max_bits = 0u;
    const size_t plane = (size_t)H * pitch;
    const float* dm = f.dmm;
    typedef float v4f __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) v4f gv4f;
    const bool vec_in = (((uintptr_t)dm | (uintptr_t)(pitch * 4)) & 15) == 0;
    const bool vec_out = (((uintptr_t)f.pts | (uintptr_t)f.nrm | (uintptr_t)(pitch * 4) | (uintptr_t)(plane * 4)) & 15) == 0 &&
                         (((uintptr_t)f.valid) & 3) == 0;
    const int p0 = c * kValidChunk + 4 * (int)threadIdx.x;
    int cnt = 0;
    if (p0 < npx) {
        const int y = p0 / W, x0 = p0 - y * W;
        if (x0 + 3 < W) {
            const uint32_t ys[3] = {(uint32_t)max(y - 1, 0), (uint32_t)y, (uint32_t)min(y + 1, H - 1)};
            const uint32_t xl = (uint32_t)max(x0 - 1, 0), xr = (uint32_t)min(x0 + 4, W - 1);
            float win[3][6];
            const bool v4 = vec_in && (x0 & 3) == 0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const uint32_t r = ys[j] * (uint32_t)pitch;
                win[j][0] = plane_ld(dm, r + xl);
                if (v4) {
                    const v4f m = *(const gv4f*)((const gbyte*)dm + (r + (uint32_t)x0) * 4u);
                    win[j][1] = m[0]; win[j][2] = m[1]; win[j][3] = m[2]; win[j][4] = m[3];
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) win[j][1 + i] = plane_ld(dm, r + (uint32_t)(x0 + i));
                }
                win[j][5] = plane_ld(dm, r + xr);
            }
            float px[4], py[4], pz[4], n0[4], n1[4], n2[4];
            uint32_t flags = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float nb[3][3];
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int i = 0; i < 3; ++i) nb[j][i] = win[j][k + i];
                const uint8_t fl = normal_pixel(f, x0 + k, y, nb, px[k], py[k], pz[k], n0[k], n1[k], n2[k]);
                flags |= (uint32_t)fl << (8 * k);
                cnt += fl & 1;
            }
            const uint32_t o = (uint32_t)y * (uint32_t)pitch + (uint32_t)x0;
            if (vec_out && (x0 & 3) == 0) {
                *(gv4f*)((gbyte*)f.pts + o * 4u) = v4f{px[0], px[1], px[2], px[3]};
                *(gv4f*)((gbyte*)(f.pts + plane) + o * 4u) = v4f{py[0], py[1], py[2], py[3]};
                *(gv4f*)((gbyte*)(f.pts + 2 * plane) + o * 4u) = v4f{pz[0], pz[1], pz[2], pz[3]};
                *(gv4f*)((gbyte*)f.nrm + o * 4u) = v4f{n0[0], n0[1], n0[2], n0[3]};
                *(gv4f*)((gbyte*)(f.nrm + plane) + o * 4u) = v4f{n1[0], n1[1], n1[2], n1[3]};
                *(gv4f*)((gbyte*)(f.nrm + 2 * plane) + o * 4u) = v4f{n2[0], n2[1], n2[2], n2[3]};
                *(__attribute__((address_space(1))) uint32_t*)((gbyte*)f.valid + o) = flags;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    *plane_at(f.pts, o + k) = px[k];
                    *plane_at(f.pts + plane, o + k) = py[k];
                    *plane_at(f.pts + 2 * plane, o + k) = pz[k];
                    *plane_at(f.nrm, o + k) = n0[k];
                    *plane_at(f.nrm + plane, o + k) = n1[k];
                    *plane_at(f.nrm + 2 * plane, o + k) = n2[k];
                    *plane_at(f.valid, o + k) = (uint8_t)(flags >> (8 * k));
                }
            }
        } else {
            // the 4 pixels wrap to the next row (or end the frame): one at a time
            for (int k = 0; k < 4 && p0 + k < npx; ++k) {
                const int yk = (p0 + k) / W, xk = p0 + k - yk * W;
                const uint32_t xs[3] = {(uint32_t)max(xk - 1, 0), (uint32_t)xk, (uint32_t)min(xk + 1, W - 1)};
                const uint32_t ys[3] = {(uint32_t)max(yk - 1, 0), (uint32_t)yk, (uint32_t)min(yk + 1, H - 1)};
                float nb[3][3];
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int i = 0; i < 3; ++i) nb[j][i] = plane_ld(dm, ys[j] * (uint32_t)pitch + xs[i]);
                float px, py, pz, n0, n1, n2;
                const uint8_t fl = normal_pixel(f, xk, yk, nb, px, py, pz, n0, n1, n2);
                const uint32_t o = (uint32_t)yk * (uint32_t)pitch + (uint32_t)xk;
                *plane_at(f.pts, o) = px;
                *plane_at(f.pts + plane, o) = py;
                *plane_at(f.pts + 2 * plane, o) = pz;
                *plane_at(f.nrm, o) = n0;
                *plane_at(f.nrm + plane, o) = n1;
                *plane_at(f.nrm + 2 * plane, o) = n2;
                *plane_at(f.valid, o) = fl;
                cnt += fl & 1;
            }
        }
    }
    if (count) {
        cnt = block_sum(cnt, sh);
        if (threadIdx.x == 0) f.chunk_cnt[c] = cnt;
    }
}

// ------------------------------------------------------------------ valid list
// Row-major list L of depth-valid pixels (the fixed per-frame point set the
// sampler indexes) plus the round-0 point list; labels start at -1.
// The scoring list walks the image in 8x8-pixel blocks (blocks in row-major
// order, pixels row-major inside a block) so that 64 consecutive points are
// close in space; the sampling list L stays row-major.  Scan position q of the
// padded block grid maps to pixel (x, y), outside the image past the edges.
// The round-0 list holds every scan position (a pixel without a point is a
// NaN entry), so it needs no compaction; later rounds compact.
__device__ __forceinline__ int scan_positions(const FrameDev& f) {
    return ((f.W + kScanBlock - 1) / kScanBlock) * ((f.H + kScanBlock - 1) / kScanBlock) * kScanBlock * kScanBlock;
}

__device__ __forceinline__ bool scan_pixel(const FrameDev& f, int q, int& x, int& y) {
    constexpr int B2 = kScanBlock * kScanBlock;
    const int bw = (f.W + kScanBlock - 1) / kScanBlock;
    const int b = q / B2, w = q - b * B2;
    const int by = b / bw, bx = b - by * bw;
    x = bx * kScanBlock + w % kScanBlock;
    y = by * kScanBlock + w / kScanBlock;
    return x < f.W && y < f.H && q < scan_positions(f);
}

__global__ __launch_bounds__(kBlock) void k_valid_count(const FrameDev* __restrict__ tab) {
    __shared__ int sh[4];
    const FrameDev& f = tab[blockIdx.z];
    const int npx = f.W * f.H;
    const int nch = (npx + kValidChunk - 1) / kValidChunk;
    if (blockIdx.x == 0 && threadIdx.x == 0) f.st->p1max_bits = 0u;
    static_assert(kValidChunk == 4 * kBlock, "four pixels per thread and chunk");
    const gu8_cptr vg = (gu8_cptr)f.valid;
    const bool word_rows = ((f.pitch | (int)(uintptr_t)f.valid) & 3) == 0;
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        // pixels p0..p0+3: one 32-bit load where they share a row, bytes otherwise
        const int p0 = c * kValidChunk + 4 * (int)threadIdx.x;
        int cnt = 0;
        if (p0 < npx) {
            const int y = p0 / f.W, x = p0 - y * f.W;
            if (word_rows && x + 3 < f.W && (x & 3) == 0) {
                const uint32_t w = *(const __attribute__((address_space(1))) uint32_t*)(vg + (size_t)y * f.pitch + x);
                cnt = __popc(w & 0x01010101u);
            } else {
                for (int i = 0; i < 4 && p0 + i < npx; ++i) {
                    const int yy = (p0 + i) / f.W, xx = p0 + i - yy * f.W;
                    cnt += vg[(size_t)yy * f.pitch + xx] & 1;
                }
            }
        }
        cnt = block_sum(cnt, sh);
        if (threadIdx.x == 0) f.chunk_cnt[c] = cnt;
    }
}

__global__ __launch_bounds__(kBlock) void k_valid_scatter(const FrameDev* __restrict__ tab) {
    __shared__ int sh[8];
    __shared__ int s_off[kValidChunk];
    const FrameDev& f = tab[blockIdx.z];
    const int npx = f.W * f.H;
    const int nch = (npx + kValidChunk - 1) / kValidChunk;
    // for every 4 row-major pixels p .. p + 3 (p a multiple of 4), the number of
    // depth-valid pixels before p: a pixel's valid-list position is that plus the
    // valid ones before it among the 4 (the diffusion ping-pong buffer is free by now)
    int32_t* __restrict__ qpre = reinterpret_cast<int32_t*>(f.delta[0]);
    const gu8_cptr vg = (gu8_cptr)f.valid;
    const gi32_cptr ccnt = (gi32_cptr)f.chunk_cnt;
    // flags and labels of 4 pixels of one row as one 32-bit word where rows allow it
    const bool words = (((uintptr_t)f.valid | (uintptr_t)f.labels | (uintptr_t)f.pitch) & 3) == 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // valid pixels before chunk c, carried from this block's previous chunk
    // a block takes a contiguous run of chunks: the valid pixels before its first chunk are
    // summed once, then carried from chunk to chunk
    const int per = (nch + (int)gridDim.x - 1) / (int)gridDim.x;
    const int c0 = (int)blockIdx.x * per, c1 = min(nch, c0 + per);
    if (c0 >= nch) return;  // the whole block
    int before = 0;
    {
        int add = 0;
        for (int i = threadIdx.x; i < c0; i += kBlock) add += ccnt[i];
        before = block_sum(add, sh);
    }
    for (int c = c0; c < c1; ++c) {
        // pixels p0 .. p0 + 3 (row-major), 4 per thread
        const int p0 = c * kValidChunk + 4 * (int)threadIdx.x;
        const int y0 = p0 / f.W, x0 = p0 - y0 * f.W;
        const bool row4 = p0 + 3 < npx && x0 + 3 < f.W;
        int off[4];
        int bits = 0;
        if (row4) {
            const int o = y0 * f.pitch + x0;
#pragma unroll
            for (int j = 0; j < 4; ++j) off[j] = o + j;
            if (words) {
                const uint32_t w = *(const __attribute__((address_space(1))) uint32_t*)(vg + o);
                bits = (int)((w & 1u) | ((w >> 7) & 2u) | ((w >> 14) & 4u) | ((w >> 21) & 8u));
                *reinterpret_cast<uint32_t*>(f.labels + o) = 0xFFFFFFFFu;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    bits |= (vg[o + j] & 1) << j;
                    f.labels[o + j] = -1;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int p = min(p0 + j, npx - 1);
                const int y = p / f.W, x = p - y * f.W;
                off[j] = y * f.pitch + x;
                if (p0 + j < npx) {
                    bits |= (vg[off[j]] & 1) << j;
                    f.labels[off[j]] = -1;
                }
            }
        }
        // row-major ranks: the valid pixels of lower lanes and waves, then this thread's lower ones
        unsigned long long m[4];
        int below = 0, wtot = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            m[j] = __ballot((bits >> j) & 1);
            below += __popcll(m[j] & lanemask_lt());
            wtot += __popcll(m[j]);
        }
        if (lane == 0) sh[4 + wave] = wtot;  // block_sum uses sh[0..3]
        __syncthreads();
        int base = before + below, tot = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            base += w < wave ? sh[4 + w] : 0;
            tot += sh[4 + w];
        }
        if (p0 < npx) qpre[p0 >> 2] = base;
        int kk[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            kk[j] = (bits >> j) & 1 ? base : -1;
            base += (bits >> j) & 1;
        }
        // the chunk's entries of L through LDS, so that consecutive lanes store consecutive entries
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (kk[j] >= 0) s_off[kk[j] - before] = off[j];
        __syncthreads();
        for (int i = threadIdx.x; i < tot; i += kBlock) {
            f.L[before + i] = s_off[i];
            f.taken[before + i] = 0;
            if (f.dbg.valid_list) f.dbg.valid_list[before + i] = s_off[i];
        }
        __syncthreads();  // the next chunk rewrites sh[4..7] and s_off
        const int run = before + tot;
        before = run;
        if (c == nch - 1 && threadIdx.x == 0) {
            RoundState* st = f.st;
            st->M0 = run;
            st->round[0].M = run;
            st->round[0].Mlen = scan_positions(f);
            st->round[0].active = (run >= 3 && f.max_planes >= 1) ? 1 : 0;
            for (int r = 1; r <= kMaxRounds; ++r) st->round[r].active = 0;
            f.n_planes[0] = 0;
            if (f.dbg.n_valid) f.dbg.n_valid[0] = run;
        }
    }
}

// ------------------------------------------------------------------ hypotheses
// The random choice of 3 points in Alg. 2: word w of Philox block
// (j, r, b, 0) under key (seed, frame) picks list position floor(w * M0 / 2^64);
// it is skipped if that pixel is already assigned or already chosen; 16
// blocks at most.  The list L is fixed per frame, so the draws of round r do
// not depend on how many points earlier rounds removed.
// 16 lanes per hypothesis compute its 16 Philox blocks at once and look up
// their 64 candidates in the per-position assignment bytes, which the
// removal sets with plain byte stores (a bitmap would need atomic ORs, which
// contend on shared words).
constexpr int kHypLanes = 16;
constexpr int kHypPerBlock = kBlock / kHypLanes;

// Read through the global address space: a generic (flat) load may alias LDS,
// so the compiler would not issue the next one before the preceding LDS store.
__device__ __forceinline__ bool point_taken(const FrameDev& f, int k) { return ((gu8_cptr)f.taken)[k] != 0; }
__device__ __forceinline__ int list_pixel(const FrameDev& f, int k) { return ((gi32_cptr)f.L)[k]; }
__device__ __forceinline__ float3 load_point_g(const FrameDev& f, int off) {
    const size_t plane = (size_t)f.H * f.pitch;
    const gf32_cptr p = (gf32_cptr)f.pts;
    return make_float3(p[off], p[plane + off], p[2 * plane + off]);
}

// Floats as integers of the same order (the sign-magnitude bits of negative
// values flipped), so that min / max over a wave are integer DPP min / max.
__device__ __forceinline__ int ordered_bits(float v) {
    const int b = __float_as_int(v);
    return b ^ ((b >> 31) & 0x7FFFFFFF);
}
__device__ __forceinline__ float from_ordered_bits(int b) { return __int_as_float(b ^ ((b >> 31) & 0x7FFFFFFF)); }

// min / max over the wave with DPP lane permutes (no LDS): pairs, quads, rows
// of 16 by rotation, then the row broadcasts; lane 63 ends with the result.
template <bool MAX>
__device__ __forceinline__ int wave_extreme_to_lane63(int v) {
    v = dpp_ext<MAX, 0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_ext<MAX, 0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_ext<MAX, 0x124>(v);  // row_ror:4
    v = dpp_ext<MAX, 0x128>(v);  // row_ror:8
    v = dpp_ext<MAX, 0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_ext<MAX, 0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

__device__ __forceinline__ int align64(int n) { return (n + 63) & ~63; }

// The padding entry of a point list: NaN coordinates, which no residual test
// passes, so padding is never an inlier, never kept, and never in a box.
__device__ __forceinline__ float4 pad_point() {
    const float qnan = __int_as_float(0x7fc00000);
    return make_float4(qnan, qnan, qnan, __int_as_float(-1));
}

// min / max over each row of 16 lanes (quad permutes and row rotations):
// every lane of the row ends with the row's result.
template <bool MAX>
__device__ __forceinline__ int row_extreme(int v) {
    v = dpp_ext<MAX, 0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_ext<MAX, 0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_ext<MAX, 0x124>(v);  // row_ror:4
    v = dpp_ext<MAX, 0x128>(v);  // row_ror:8
    return v;
}
__device__ __forceinline__ int row_sum(int v) {
    v = dpp_add<0xB1>(v);
    v = dpp_add<0x4E>(v);
    v = dpp_add<0x124>(v);
    v = dpp_add<0x128>(v);
    return v;
}

// Bounding boxes of ntiles consecutive 64-point tiles of a list held at src
// (LDS or global memory the block has written), over their points that are
// not padding: box[2 t] = centre (w: their count as integer bits), box[2 t +
// 1] = half extents.  The calling wave takes tiles in groups of 4 (group g,
// g + step, ...): a 16-lane row per tile, 4 consecutive points per lane,
// reduced first in the lane (float min / max, which pass over NaN), then
// across the row as order-preserving integers (each permute folds into its
// v_min_i32_dpp / v_max_i32_dpp).
__device__ __forceinline__ void tile_boxes(const float4* src, int ntiles, float4* box, int g, int step) {
    const int lane = threadIdx.x & 63, row = lane >> 4, i = lane & 15;
    for (; g * 4 < ntiles; g += step) {
        const int tile = g * 4 + row;
        float4 q[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) q[j] = tile < ntiles ? src[tile * 64 + 4 * i + j] : pad_point();
        float lx = INFINITY, ly = INFINITY, lz = INFINITY, hx = -INFINITY, hy = -INFINITY, hz = -INFINITY;
        int n = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            lx = fminf(lx, q[j].x); ly = fminf(ly, q[j].y); lz = fminf(lz, q[j].z);
            hx = fmaxf(hx, q[j].x); hy = fmaxf(hy, q[j].y); hz = fmaxf(hz, q[j].z);
            n += q[j].x == q[j].x ? 1 : 0;
        }
        lx = from_ordered_bits(row_extreme<false>(ordered_bits(lx)));
        ly = from_ordered_bits(row_extreme<false>(ordered_bits(ly)));
        lz = from_ordered_bits(row_extreme<false>(ordered_bits(lz)));
        hx = from_ordered_bits(row_extreme<true>(ordered_bits(hx)));
        hy = from_ordered_bits(row_extreme<true>(ordered_bits(hy)));
        hz = from_ordered_bits(row_extreme<true>(ordered_bits(hz)));
        n = row_sum(n);
        if (i == 15 && tile < ntiles) {
            const float cx = 0.5f * (lx + hx), cy = 0.5f * (ly + hy), cz = 0.5f * (lz + hz);
            // the rounded differences may fall short of the true ones by an ulp: widen by 2^-20
            const float w = 1.0f + 9.5367432e-7f;
            const float ex = fmaxf(hx - cx, cx - lx) * w, ey = fmaxf(hy - cy, cy - ly) * w,
                        ez = fmaxf(hz - cz, cz - lz) * w;
            box[2 * tile] = make_float4(cx, cy, cz, __int_as_float(n));
            box[2 * tile + 1] = make_float4(ex, ey, ez, 0.f);
        }
    }
}

// The first RANSAC round's scoring list: position q of the 8x8-block scan
// holds the point of its pixel (x, y, z, its valid-list position as integer bits),
// or NaN where the pixel is outside the frame or has no depth, so the list
// needs no compaction; the boxes of its 64-point tiles (one tile per 8x8
// block) are made here, as is the frame-wide bound on |p|_1 that the matrix-core
// scorers' recheck bands use.  A block takes 16 tiles (1024 positions) per
// step, staged in LDS for the boxes.
__global__ __launch_bounds__(kBlock) void k_list0(const FrameDev* __restrict__ tab) {
    __shared__ float4 stage[kValidChunk];
    __shared__ float shf[4];
    const FrameDev& f = tab[blockIdx.z];
    const int nq = scan_positions(f);
    const int nchq = (nq + kValidChunk - 1) / kValidChunk;
    const size_t plane = (size_t)f.H * f.pitch;
    const gu8_cptr vg = (gu8_cptr)f.valid;
    const gf32_cptr pg = (gf32_cptr)f.pts;
    const gi32_cptr qpre = (gi32_cptr)f.delta[0];  // valid pixels before each row-major group of 4
    float4* __restrict__ out = f.list[0];
    // a thread takes 4 consecutive scan positions, 4 pixels of one row of one 8x8 block
    // (x0 a multiple of 4): one 16-byte load per plane where the rows allow it
    typedef float v4f __attribute__((ext_vector_type(4)));
    const bool vec_pts = (((uintptr_t)f.pts | (uintptr_t)(f.pitch * 4) | (uintptr_t)(plane * 4)) & 15) == 0;
    const bool vec_flags = (((uintptr_t)f.valid | (uintptr_t)f.pitch) & 3) == 0;
    const bool quad_rows = (f.W & 3) == 0;  // a thread's 4 pixels are then one row-major group of 4
    float p1 = 0.f;
    for (int c = blockIdx.x; c < nchq; c += gridDim.x) {
        const int q0 = c * kValidChunk + 4 * (int)threadIdx.x;
        int x0 = 0, y = 0;
        const bool in_scan = q0 < nq;
        scan_pixel(f, q0, x0, y);  // (x0, y) of position q0, possibly past the frame's edge
        const bool row_in = in_scan && y < f.H;
        const bool full = row_in && x0 + 3 < f.W;  // all 4 pixels inside the frame
        float px[4] = {0.f, 0.f, 0.f, 0.f}, py[4] = {0.f, 0.f, 0.f, 0.f}, pz[4] = {0.f, 0.f, 0.f, 0.f};
        int vb[4] = {0, 0, 0, 0}, lp[4] = {0, 0, 0, 0};
        const uint32_t o = (uint32_t)y * (uint32_t)f.pitch + (uint32_t)x0;
        if (full && vec_pts) {
            const v4f a = *(const __attribute__((address_space(1))) v4f*)(pg + o);
            const v4f b = *(const __attribute__((address_space(1))) v4f*)(pg + plane + o);
            const v4f d = *(const __attribute__((address_space(1))) v4f*)(pg + 2 * plane + o);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                px[j] = a[j];
                py[j] = b[j];
                pz[j] = d[j];
            }
        } else if (row_in) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (x0 + j < f.W) {
                    px[j] = pg[o + j];
                    py[j] = pg[plane + o + j];
                    pz[j] = pg[2 * plane + o + j];
                }
        }
        if (full && vec_flags) {
            const uint32_t w = *(const __attribute__((address_space(1))) uint32_t*)(vg + o);
#pragma unroll
            for (int j = 0; j < 4; ++j) vb[j] = (w >> (8 * j)) & 1;
        } else if (row_in) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (x0 + j < f.W) vb[j] = vg[o + j] & 1;
        }
        const int lo = y * f.W + x0;
        if (full && quad_rows) {
            int run = qpre[lo >> 2];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                lp[j] = run;
                run += vb[j];
            }
        } else if (row_in) {
            // the group of 4 may start in the previous row: its earlier pixels one by one
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (x0 + j < f.W && vb[j]) {
                    const int p = lo + j;
                    int n = qpre[p >> 2];
                    for (int i = p & ~3; i < p; ++i) {
                        const int yi = i / f.W, xi = i - yi * f.W;
                        n += vg[(size_t)yi * f.pitch + xi] & 1;
                    }
                    lp[j] = n;
                }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float4 q = pad_point();
            if (vb[j]) {
                q = make_float4(px[j], py[j], pz[j], __int_as_float(lp[j]));
                p1 = fmaxf(p1, fabsf(px[j]) + fabsf(py[j]) + fabsf(pz[j]));
            }
            stage[4 * threadIdx.x + j] = q;
        }
        __syncthreads();
        // the chunk's positions in order, one 16-byte store per thread and step
#pragma unroll
        for (int k = 0; k < kValidChunk / kBlock; ++k) {
            const int i = k * kBlock + threadIdx.x;
            if (c * kValidChunk + i < nq) out[c * kValidChunk + i] = stage[i];
        }
        const int ntiles = min(kValidChunk, nq - c * kValidChunk) >> 6;
        tile_boxes(stage, ntiles, f.tbox + 2 * (c * kValidChunk >> 6), threadIdx.x >> 6, kBlock / 64);
        __syncthreads();  // the stage is reused by the next chunk
    }
    // frame-wide bound on |p|_1 for the recheck bands of the matrix-core scorers
    // (non-negative floats order as their bit patterns)
    float pm = __int_as_float(wave_ext<true>(__float_as_int(p1)));
    if ((threadIdx.x & 63) == 0) shf[threadIdx.x >> 6] = pm;
    __syncthreads();
    if (threadIdx.x == 0) {
        pm = fmaxf(fmaxf(shf[0], shf[1]), fmaxf(shf[2], shf[3]));
        if (pm > 0.f) atomicMax(&f.st->p1max_bits, __float_as_uint(pm));
    }
}

// Workgroups go to the 8 XCDs in turn (workgroup i to XCD i mod 8), each XCD
// with its own L2.  This maps the first nblocks workgroups of a 1-D grid (nf *
// bpf blocks padded to a multiple of 8) so that each XCD takes a contiguous range of (frame, block)
// pairs, i.e. about nf / 8 whole frames, whose random lookups then share one
// L2.  False for the padding blocks.
constexpr int kXcds = 8;
__device__ __forceinline__ bool xcd_frame_block(int bpf, int nf, int nblocks, int& frame, int& bx) {
    const int T = bpf * nf;
    const int per = nblocks / kXcds;
    const int L = blockIdx.x;
    const int id = (L % kXcds) * per + L / kXcds;
    if (id >= T) return false;
    frame = id / bpf;
    bx = id - frame * bpf;
    return true;
}

// The first of this row's candidates (16 lanes, 4 each, draw order 4 b + q)
// that is still in play; its value in every lane of the row (INT_MAX: none).
// The row minima are DPP permutes within the row's 16 lanes.
__device__ __forceinline__ int row_first_candidate(const int (&cand)[4], int b) {
    int key = 64;
#pragma unroll
    for (int q = 3; q >= 0; --q)
        if (cand[q] >= 0) key = 4 * b + q;
    key = dpp_ext<false, 0xB1>(key);   // quad_perm [1,0,3,2]
    key = dpp_ext<false, 0x4E>(key);   // quad_perm [2,3,0,1]
    key = dpp_ext<false, 0x124>(key);  // row_ror:4
    key = dpp_ext<false, 0x128>(key);  // row_ror:8
    int val = 0x7FFFFFFF;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (key == 4 * b + q) val = cand[q];
    val = dpp_ext<false, 0xB1>(val);
    val = dpp_ext<false, 0x4E>(val);
    val = dpp_ext<false, 0x124>(val);
    val = dpp_ext<false, 0x128>(val);
    return val;
}

// Hypotheses of round r for the 16 hypotheses of block bx of frame f.  Each
// hypothesis is one 16-lane row: lane b draws Philox block b (4 candidate
// list positions), a candidate whose point is assigned is dropped, and the
// triple is the first three distinct candidates left in draw order, exactly
// the sequential draw's (three rounds of: the row's first candidate, then
// every copy of it dropped).
__device__ __forceinline__ void hypgen_block(const FrameDev& f, int r, int bx) {
    const RoundRec rr = round_rec(f, r);
    const uint64_t M0 = (uint64_t)((const __attribute__((address_space(4))) int32_t*)f.st)[0];  // RoundState::M0
    if (!rr.active) return;
    const int hl = threadIdx.x / kHypLanes, b = threadIdx.x % kHypLanes;
    const int j = bx * kHypPerBlock + hl;
    if (bx * kHypPerBlock >= f.hyps) return;
    static_assert(kHypLanes == 16, "one DPP row per hypothesis");
    int cand[4] = {-1, -1, -1, -1};
    if (j < f.hyps) {
        uint64_t c[4] = {(uint64_t)j, (uint64_t)r, (uint64_t)b, 0ull};
        philox4x64_10(c, f.seed, f.frame_id);
        int k[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) k[q] = (int)__umul64hi(c[q], M0);
        // the first round removes nothing before it: no lookups then
        if (rr.M != (int)M0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) k[q] = point_taken(f, k[q]) ? -1 : k[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) cand[q] = k[q];
    }
    int slot[3];
    int got = 0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int v = row_first_candidate(cand, b);
        slot[s] = v;
        got += v != 0x7FFFFFFF ? 1 : 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (cand[q] == v) cand[q] = -1;
    }
    if (b != 0 || j >= f.hyps) return;
    float4 h = make_float4(0.f, 0.f, 0.f, __int_as_float(0x7fc00000));
    float3 p0 = make_float3(0.f, 0.f, 0.f);
    if (got == 3) {
        p0 = load_point_g(f, list_pixel(f, slot[0]));
        h = plane_from_points(p0, load_point_g(f, list_pixel(f, slot[1])), load_point_g(f, list_pixel(f, slot[2])));
    }
    f.hyp[j] = h;
    f.hyp_p0[j] = make_float4(p0.x, p0.y, p0.z, 0.f);
    f.counts[j] = 0;
    f.triples[3 * j + 0] = got == 3 ? slot[0] : -1;
    f.triples[3 * j + 1] = got == 3 ? slot[1] : -1;
    f.triples[3 * j + 2] = got == 3 ? slot[2] : -1;
    if (f.dbg.hyps) reinterpret_cast<float4*>(f.dbg.hyps)[(size_t)r * f.hyps + j] = h;
    if (f.dbg.triples) {
        int32_t* t = f.dbg.triples + ((size_t)r * f.hyps + j) * 3;
        t[0] = got == 3 ? slot[0] : -1;
        t[1] = got == 3 ? slot[1] : -1;
        t[2] = got == 3 ? slot[2] : -1;
    }
}

// Planes of caller-given triples of pixel offsets (debug scoring).
__global__ __launch_bounds__(kBlock) void k_hyp_from_triples(const FrameDev* __restrict__ tab,
                                                              const int32_t* __restrict__ tri, int n) {
    const FrameDev& f = tab[0];
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    // scoring only: hyp and counts are the caller's n-entry buffers here, and no
    // refit follows, so the slot's per-hypothesis arrays (sized for one) stay untouched
    f.hyp[j] = plane_from_points(load_point(f, tri[3 * j]), load_point(f, tri[3 * j + 1]), load_point(f, tri[3 * j + 2]));
    f.counts[j] = 0;
}

// ------------------------------------------------------------------ selection
// j* = the valid hypothesis with the most inliers, the lowest index among
// equal counts; -1 if no hypothesis is valid.  Every moments block computes it.
constexpr int kSelPerThread = 4;
__device__ __forceinline__ int select_jstar(const FrameDev& f, int* sh) {
    const int H = f.hyps;
    const gf32_cptr hw = (gf32_cptr)f.hyp;  // d of hypothesis j at 4 j + 3 (NaN: invalid)
    const gi32_cptr cn = (gi32_cptr)f.counts;
    int bc = -1, bj = 0x7FFFFFFF;
    for (int j0 = threadIdx.x; j0 < H; j0 += kBlock * kSelPerThread) {
        float d[kSelPerThread];
        int cnt[kSelPerThread];
#pragma unroll
        for (int q = 0; q < kSelPerThread; ++q) {
            const int jj = min(j0 + q * kBlock, H - 1);
            d[q] = hw[4 * jj + 3];
            cnt[q] = cn[jj];
        }
#pragma unroll
        for (int q = 0; q < kSelPerThread; ++q) {
            const int j = j0 + q * kBlock;
            if (j < H && d[q] == d[q] && (cnt[q] > bc || (cnt[q] == bc && j < bj))) {
                bc = cnt[q];
                bj = j;
            }
        }
    }
    const int wc = wave_ext<true>(bc);
    const int wj = wave_ext<false>(bc == wc ? bj : 0x7FFFFFFF);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sh[w] = wc;
        sh[4 + w] = wj;
    }
    __syncthreads();
    int best = sh[0], js = sh[4];
    for (int i = 1; i < 4; ++i)
        if (sh[i] > best || (sh[i] == best && sh[4 + i] < js)) {
            best = sh[i];
            js = sh[4 + i];
        }
    return best < 0 ? -1 : js;
}

// ------------------------------------------------------------------ scoring
// count_j = #{i in R_r : |n_j . p_i + d_j| < t}.  A block owns HB hypotheses
// (uniform: scalar loads into SGPRs) and a strided share of the points, one
// point per lane in wave-uniform tiles of 64.  Each (point, hypothesis) costs
// 3 FMA and one compare on the vector ALU; the compare's lane mask is counted
// on the scalar unit (popcount + add), so the counters live in SGPRs and each
// wave adds its totals to the global counts with one integer atomic per
// hypothesis (order-free).
template <int HB>
__device__ __forceinline__ void score_block(const FrameDev& f, int r, int M) {
    const int h0 = blockIdx.y * HB;
    if (h0 >= f.hyps) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float4* __restrict__ pts = f.list[r & 1];
    float4 h[HB];
#pragma unroll
    for (int i = 0; i < HB; ++i) h[i] = (h0 + i < f.hyps) ? f.hyp[h0 + i] : make_float4(0.f, 0.f, 0.f, __int_as_float(0x7fc00000));
    const float t = f.thresh;
    uint32_t cnt[HB];
#pragma unroll
    for (int i = 0; i < HB; ++i) cnt[i] = 0u;
    const float qnan = __int_as_float(0x7fc00000);
    const int stride = gridDim.x * kBlock;
    int base = blockIdx.x * kBlock + wave * 64;
    float4 pn = make_float4(qnan, qnan, qnan, 0.f);  // the next tile's point, loaded one iteration ahead
    if (base + lane < M) pn = pts[base + lane];
    for (; base < M; base += stride) {
        const float4 p = pn;
        pn = make_float4(qnan, qnan, qnan, 0.f);
        if (base + stride + lane < M) pn = pts[base + stride + lane];
#pragma unroll
        for (int k = 0; k < HB; ++k)
            cnt[k] += (uint32_t)__popcll(__ballot(fabsf(canon_res(h[k], p.x, p.y, p.z)) < t));
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < HB; ++k)
            if (cnt[k] != 0u && h0 + k < f.hyps) atomicAdd(&f.counts[h0 + k], (int)cnt[k]);
    }
}

template <int HB>
__global__ __launch_bounds__(kBlock) void k_score(const FrameDev* __restrict__ tab, int r) {
    const FrameDev& f = tab[blockIdx.z];
    const RoundRec rr = round_rec(f, r);
    if (!rr.active) return;
    score_block<HB>(f, r, rr.Mlen);
}

// ------------------------------------------------------------------ culled scoring
// Loads through the global address space (global_load rather than the
// generic flat path).  Only for data no kernel of the same launch writes.
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) v4f_t* gv4_ptr;

__device__ __forceinline__ float4 ld_global4(const float4* p, int i) {
    const v4f_t v = ((gv4_ptr)p)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

// x, y, z of a float4 record (a 12-byte load: w is never read)
typedef float v3f_t __attribute__((ext_vector_type(3)));
__device__ __forceinline__ float3 ld_global_xyz(const float4* p, int i) {
    const v3f_t v = *reinterpret_cast<const __attribute__((address_space(1))) v3f_t*>(
        reinterpret_cast<const __attribute__((address_space(1))) char*>((gv4_ptr)p) + (size_t)i * 16);
    return make_float3(v.x, v.y, v.z);
}


// The start of round r: the hypotheses, over an XCD-aware 1-D mapping of
// (frame, block) pairs.  They read only what the previous round's removal
// left (the tile boxes of the round's list were made with the list).
__global__ __launch_bounds__(kBlock) void k_round_start(const FrameDev* __restrict__ tab, int r, int bpf, int nf) {
    int frame, bx;
    if (xcd_frame_block(bpf, nf, (int)gridDim.x, frame, bx)) hypgen_block(tab[frame], r, bx);
}

// Inlier counts over 64-point tiles (Eq. 3, Alg. 2): the tile boxes decide
// most (tile, hypothesis) pairs; the rest are counted point by point.
//
// A block holds 64 Q hypotheses, Q per lane; its four waves take tiles in
// turn.  For each tile every lane bounds its hypotheses' residuals over the
// tile's box: |n.c + d| -/+ (|nx| ex + |ny| ey + |nz| ez).  With a margin of
// 16 u (P1 + |d|) (u = 2^-24, P1 = max |p|_1 of the frame), which exceeds the
// FP32 rounding of the bound and of the canonical residual, a tile lies
// wholly outside (no inliers) or wholly inside (all its points are inliers)
// exactly as the canonical formula decides.  The hypotheses left straddling
// the tile are evaluated on its points, so every count is the canonical one:
//  - a few of them (or every one, for PP_SCORE_FP32): one at a time with the
//    canonical formula, the tile's points one per lane (straddle_loop);
//  - otherwise on the matrix cores, 16 at a time (mfma_groups).
// A tile reaches the matrix cores when at least max(40, 3/8 of the block's)
// hypotheses straddle it; fewer go through straddle_loop, which costs less per
// straddler than a 16-hypothesis group on the matrix cores plus its compares.
constexpr int mfma_min_straddlers(int nh) { return 3 * nh / 8 > 40 ? 3 * nh / 8 : 40; }

// One tile's straddling hypotheses S (bit k: slot k of hyp_lds) against the
// tile's points (one per lane; lanes past the list's end hold a NaN point,
// which no hypothesis takes as an inlier), lowest first.  Each straddler
// occurs once per tile: its count is written straight into its lane of the
// result (v_writelane, lane select in M0).  S != 0.  (Reading the next
// plane ahead added more copies than it hid latency: enough waves share a
// SIMD to cover the LDS read.)
__device__ __forceinline__ int straddle_loop(unsigned long long S, const float4* hyp_lds, float3 p, float t) {
    int w = 0;
    do {
        const int k = __builtin_ctzll(S);
        asm("s_bitset0_b64 %0, %1" : "+s"(S) : "s"(k));
        // the LDS byte offset formed by one vector shift (a scalar shift and a copy otherwise)
        int off;
        asm("v_lshlrev_b32 %0, 4, %1" : "=v"(off) : "s"(k));
        const float4 h = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(hyp_lds) + off);
        const int m = __popcll(__ballot(fabsf(canon_res(h, p.x, p.y, p.z)) < t));
        asm("v_writelane_b32 %0, %2, %1" : "+v"(w) : "{m0}"(k), "s"(m));
    } while (S);
    return w;
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

// Low-precision matrix operands: 8 elements per lane (K = 32).
template <int PREC> struct LpVec { typedef bf16x8_t type; typedef __bf16 elem; };
template <> struct LpVec<PP_SCORE_FP16> { typedef f16x8_t type; typedef _Float16 elem; };

// FP16 operands carry q scaled by 2^6 (exact), so that coordinates down to
// about 1e-6 m stay normal FP16 numbers; residuals and thresholds scale alike.
template <int PREC> constexpr float lp_scale() { return PREC == PP_SCORE_FP16 ? 64.f : 1.f; }

// A value v in the low precision as hi + lo, both rounded to nearest
// (v - hi is exact in FP32), so that hi + lo is v to about u_lp^2.
template <int PREC>
__device__ __forceinline__ void lp_split(float v, typename LpVec<PREC>::elem& hi, typename LpVec<PREC>::elem& lo) {
    typedef typename LpVec<PREC>::elem lp_t;
    hi = (lp_t)v;
    lo = (lp_t)(v - (float)hi);
}

// The K elements of a low-precision operand row, in split form: lanes 0-15
// carry elements 0-7 and lanes 16-31 element 8 (K positions 0-8 of 32).
// Points: (qx_h, qy_h, qz_h, qx_l, qy_l, qz_l, qx_h, qy_h | qz_h);
// normals: (nx_h, ny_h, nz_h, nx_h, ny_h, nz_h, nx_l, ny_l | nz_l): the
// contraction is q_h.n_h + q_l.n_h + q_h.n_l, i.e. (q_h + q_l).(n_h + n_l)
// without q_l.n_l.
template <int PREC>
__device__ __forceinline__ void lp_point_row(float qx, float qy, float qz, typename LpVec<PREC>::type& row,
                                             typename LpVec<PREC>::elem& row8) {
    typename LpVec<PREC>::elem xh, xl, yh, yl, zh, zl;
    lp_split<PREC>(qx, xh, xl);
    lp_split<PREC>(qy, yh, yl);
    lp_split<PREC>(qz, zh, zl);
    row = typename LpVec<PREC>::type{xh, yh, zh, xl, yl, zl, xh, yh};
    row8 = zh;
}
template <int PREC>
__device__ __forceinline__ void lp_normal_row(float nx, float ny, float nz, typename LpVec<PREC>::type& row,
                                              typename LpVec<PREC>::elem& row8) {
    typename LpVec<PREC>::elem xh, xl, yh, yl, zh, zl;
    lp_split<PREC>(nx, xh, xl);
    lp_split<PREC>(ny, yh, yl);
    lp_split<PREC>(nz, zh, zl);
    row = typename LpVec<PREC>::type{xh, yh, zh, xh, yh, zh, xl, yl};
    row8 = zl;
}

// The straddlers of one tile on the matrix cores, 16 hypotheses a group.
// The queue qs holds their slots in s_h; sp holds the tile's 64 points
// (NaN coordinates past the list's end).  v_mfma_f32_16x16x*: 16 points
// along M (A rows), the group's 16 hypotheses along N (B columns); lane l
// holds D[4 (l/16) + v][l % 16] of each 16-point block b, so after the
// tile's four blocks every lane has 16 residuals of one hypothesis.
//   PP_SCORE_MFMA_F32: A = (x, y, z, 1), B = (nx, ny, nz, d) (16x16x4 f32);
//     D and the canonical residual differ by rounding only: at most
//     16 u (P1 + |d|) (u = 2^-24; P1 bounds |p|_1 over the tile's points).
//   PP_SCORE_BF16 / FP16 (16x16x32): A = q = p - c (c: the tile box's
//     centre) and B = n in the split form of lp_point_row / lp_normal_row
//     (unit roundoff u_lp = 2^-8 / 2^-11, staged in LDS: spa per point,
//     shb per hypothesis), C = a = n.c + d in FP32; the products are exact
//     and accumulate in FP32.  With |q_k| <= e_k and E = sum |n_k| e_k, D
//     differs from the canonical residual by at most (3 u_lp^2 + 12 u) E +
//     48 u (P1 + |d|), plus 6.2e-5 (e_x + e_y + e_z + 3 / 2^6) should the
//     matrix cores flush FP16 subnormals.
// A residual whose |D| lies farther than the band from t decides as the
// canonical one does; one inside the band (within max(recheck_band_m, the
// bound) of t) is recomputed canonically.  Counts go to LDS (ds_add).
template <int PREC>
__device__ __forceinline__ void mfma_groups(int ns, const int* __restrict__ qs, const float4* __restrict__ sp,
                                            const typename LpVec<PREC>::type* __restrict__ spa,
                                            const typename LpVec<PREC>::elem* __restrict__ spa8,
                                            const float4* __restrict__ s_h,
                                            const typename LpVec<PREC>::type* __restrict__ shb,
                                            const typename LpVec<PREC>::elem* __restrict__ shb8, int* s_cnt,
                                            float4 c, float4 e, float t, float P1, float band_min) {
    typedef typename LpVec<PREC>::type lpv_t;
    typedef typename LpVec<PREC>::elem lp_t;
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
    const float u = 5.9604645e-8f;
    const float qnan = __int_as_float(0x7fc00000);
    constexpr bool F32 = PREC == PP_SCORE_MFMA_F32;
    constexpr float S = lp_scale<PREC>();
    const lp_t z = (lp_t)0.f;
    const lpv_t zv = {z, z, z, z, z, z, z, z};
    // A operands of the tile's four 16-point blocks
    float a32[4];
    lpv_t alp[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if constexpr (F32) {
            a32[b] = reinterpret_cast<const float*>(sp + 16 * b + col)[grp];
        } else {
            alp[b] = zv;
            if (grp == 0) alp[b] = spa[16 * b + col];
            else if (grp == 1) alp[b][0] = spa8[16 * b + col];
        }
    }
    const float ulp = PREC == PP_SCORE_BF16 ? 0.00390625f : 0.00048828125f;
    const float coef = 3.f * ulp * ulp + 12.f * u;
    const float flush = PREC == PP_SCORE_FP16 ? 6.2e-5f * (e.x + e.y + e.z + 3.f / 64.f) : 0.f;
    for (int g = 0; g * 16 < ns; ++g) {
        const int k = g * 16 + col;
        const int slot = k < ns ? qs[k] : -1;
        const float4 h = slot >= 0 ? s_h[slot] : make_float4(0.f, 0.f, 0.f, qnan);
        float band = F32 ? 16.f * u * (P1 + fabsf(h.w))
                         : fmaf(coef, fmaf(fabsf(h.x), e.x, fmaf(fabsf(h.y), e.y, fabsf(h.z) * e.z)),
                                48.f * u * (P1 + fabsf(h.w))) + flush;
        band = fmaxf(band, band_min);
        const float tlo = (t - band) * S, thi = (t + band) * S;
        f32x4_t D[4];
        if constexpr (F32) {
            // component grp of the column's plane, read straight from LDS
            const float bop = slot >= 0 ? reinterpret_cast<const float*>(s_h + slot)[grp] : qnan;
            const f32x4_t zf = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int b = 0; b < 4; ++b) D[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a32[b], bop, zf, 0, 0, 0);
        } else {
            lpv_t bv = zv;
            if (slot >= 0) {
                if (grp == 0) bv = shb[slot];
                else if (grp == 1) bv[0] = shb8[slot];
            }
            const float a = fmaf(h.x, c.x, fmaf(h.y, c.y, fmaf(h.z, c.z, h.w))) * S;
            const f32x4_t cc = {a, a, a, a};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if constexpr (PREC == PP_SCORE_BF16)
                    D[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alp[b], bv, cc, 0, 0, 0);
                else
                    D[b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(alp[b], bv, cc, 0, 0, 0);
            }
        }
        // definite inliers counted; residuals inside the band only flag the wave
        int cnt = 0;
        unsigned long long amb = 0ull;
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float x = fabsf(D[b][v]);
                const bool sure = x < tlo;
                cnt += sure ? 1 : 0;
                amb |= __ballot(x < thi) & ~__ballot(sure);
            }
        if (__builtin_expect(amb != 0ull, 0)) {  // the canonical residual decides inside the band
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float x = fabsf(D[b][v]);
                    if (x >= tlo && x < thi) {
                        const float4 p = sp[16 * b + 4 * grp + v];
                        cnt += fabsf(canon_res(h, p.x, p.y, p.z)) < t ? 1 : 0;
                    }
                }
        }
        // the four lanes of a column add into its hypothesis' count
        if (slot >= 0 && cnt != 0) atomicAdd(&s_cnt[slot], cnt);
    }
}

template <int PREC, int Q>
__global__ __launch_bounds__(kBlock) void k_score_tiles(const FrameDev* __restrict__ tab, int r) {
    constexpr int NH = 64 * Q;
    constexpr bool MF = PREC != PP_SCORE_FP32;
    __shared__ float4 s_h[NH];
    __shared__ int s_cnt[NH];
    constexpr bool LP = PREC == PP_SCORE_BF16 || PREC == PP_SCORE_FP16;
    typedef typename LpVec<PREC>::type lpv_t;
    typedef typename LpVec<PREC>::elem lp_t;
    __shared__ int s_q[MF ? kBlock / 64 : 1][MF ? NH : 1];        // per wave: slots of the tile's straddlers
    __shared__ float4 s_p[MF ? kBlock / 64 : 1][MF ? 64 : 1];    // per wave: the tile's points
    __shared__ lpv_t s_pa[LP ? kBlock / 64 : 1][LP ? 64 : 1];    // per wave: split low-precision rows of q
    __shared__ lp_t s_pa8[LP ? kBlock / 64 : 1][LP ? 64 : 1];
    __shared__ lpv_t s_hb[LP ? NH : 1];                            // split low-precision rows of the normals
    __shared__ lp_t s_hb8[LP ? NH : 1];
    const FrameDev& f = tab[blockIdx.z];
    const RoundRec rr = round_rec(f, r);
    if (!rr.active) return;
    const int M = rr.Mlen;  // a multiple of 64; padding points are NaN
    const int hyps = __builtin_amdgcn_readfirstlane(f.hyps);
    const int h0 = blockIdx.y * NH;
    if (h0 >= hyps) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float qnan = __int_as_float(0x7fc00000);
    for (int j = threadIdx.x; j < NH; j += kBlock) {
        const float4 h = h0 + j < hyps ? ld_global4(f.hyp, h0 + j) : make_float4(0.f, 0.f, 0.f, qnan);
        s_h[j] = h;
        s_cnt[j] = 0;
        if constexpr (LP) lp_normal_row<PREC>(h.x, h.y, h.z, s_hb[j], s_hb8[j]);
    }
    __syncthreads();
    const float t = f.thresh;
    const float P1 = __uint_as_float(f.st->p1max_bits);
    const float u = 5.9604645e-8f;
    float4 hl[Q];
    bool hv[Q];
    float ax[Q], ay[Q], az[Q], tlo[Q], thi[Q];
    uint32_t cnt[Q];
    int w[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        hl[q] = s_h[q * 64 + lane];
        hv[q] = hl[q].w == hl[q].w;
        const float band = 16.f * u * (P1 + fabsf(hl[q].w));
        tlo[q] = t - band;
        thi[q] = t + band;
        ax[q] = fabsf(hl[q].x);
        ay[q] = fabsf(hl[q].y);
        az[q] = fabsf(hl[q].z);
        cnt[q] = 0u;
        w[q] = 0;
    }
    const float4* pts = f.list[r & 1];
    const float4* box = f.tbox;
    const int ntiles = (M + 63) >> 6;
    // each wave's next tile (box and this lane's point) is loaded one iteration ahead
    const int tstride = gridDim.x * 4;
    int tile = blockIdx.x * 4 + wave;
    float4 c_next = make_float4(0.f, 0.f, 0.f, 0.f), e_next = c_next;
    float3 p_next = make_float3(0.f, 0.f, 0.f);
    if (tile < ntiles) {
        c_next = ld_global4(box, 2 * tile);
        e_next = ld_global4(box, 2 * tile + 1);
        p_next = ld_global_xyz(pts, min(tile * 64 + lane, M - 1));
    }
    uint32_t n_tiles = 0, n_straddle = 0, n_mfma = 0;  // this wave's tiles, undecided pairs, those on the matrix cores
    for (; tile < ntiles; tile += tstride) {
        const float4 c = c_next, e = e_next;
        float3 p = p_next;
        if (tile + tstride < ntiles) {
            c_next = ld_global4(box, 2 * (tile + tstride));
            e_next = ld_global4(box, 2 * (tile + tstride) + 1);
            p_next = ld_global_xyz(pts, min((tile + tstride) * 64 + lane, M - 1));
        }
        if (__float_as_int(c.w) == 0) continue;  // a tile of padding only (no point of its 8x8 block)
        ++n_tiles;
        unsigned long long S[Q];
        int ns = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float a = fabsf(fmaf(hl[q].x, c.x, fmaf(hl[q].y, c.y, fmaf(hl[q].z, c.z, hl[q].w))));
            const float ext = fmaf(ax[q], e.x, fmaf(ay[q], e.y, az[q] * e.z));
            const bool in = hv[q] && a + ext < tlo[q];
            const bool out = !hv[q] || a - ext >= thi[q];
            cnt[q] += in ? (uint32_t)__float_as_int(c.w) : 0u;
            S[q] = __ballot(!in && !out);
            ns += __popcll(S[q]);
        }
        if (ns == 0) continue;
        n_straddle += ns;
        if (!MF || ns < mfma_min_straddlers(NH)) {
            asm volatile("" : "+v"(p.x), "+v"(p.y), "+v"(p.z));  // keeps the select out of the loops below
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (S[q]) w[q] += straddle_loop(S[q], s_h + q * 64, p, t);
            continue;
        }
        if constexpr (MF) {
            n_mfma += ns;
            // the tile's points and the straddlers' slots (in slot order); one
            // wave's LDS accesses complete in order, so no barrier is needed
            s_p[wave][lane] = make_float4(p.x, p.y, p.z, 1.f);
            if constexpr (LP) {
                constexpr float S = lp_scale<PREC>();
                lp_point_row<PREC>((p.x - c.x) * S, (p.y - c.y) * S, (p.z - c.z) * S, s_pa[wave][lane],
                                   s_pa8[wave][lane]);
            }
            int base = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                if ((S[q] >> lane) & 1ull) s_q[wave][base + __popcll(S[q] & lanemask_lt())] = q * 64 + lane;
                base += __popcll(S[q]);
            }
            // the tile's points have |p|_1 <= |c|_1 + |e|_1: the bands' bound on |p|_1 (widened by 2^-20
            // for the rounding of the sum), tighter than the frame's
            const float P1t = fminf(P1, (fabsf(c.x) + fabsf(c.y) + fabsf(c.z) + (e.x + e.y + e.z)) * 1.00000095f);
            mfma_groups<PREC>(ns, s_q[wave], s_p[wave], s_pa[LP ? wave : 0], s_pa8[LP ? wave : 0], s_h, s_hb, s_hb8,
                              s_cnt, c, e, t, P1t, f.band);
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int v = (int)cnt[q] + w[q];
        if (v) atomicAdd(&s_cnt[q * 64 + lane], v);
    }
    if (f.dbg.scored && lane == 0 && n_tiles) {
        const uint32_t nvalid = (uint32_t)min(NH, hyps - h0);
        atomicAdd(f.dbg.scored, (unsigned long long)n_tiles * nvalid - n_straddle);
        atomicAdd(f.dbg.scored + 1, 64ull * n_straddle);
        if (n_mfma) atomicAdd(f.dbg.scored + 2, 64ull * n_mfma);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < NH; j += kBlock) {
        const int v = s_cnt[j];
        if (v && h0 + j < hyps) atomicAdd(&f.counts[h0 + j], v);
    }
}

// ------------------------------------------------------------------ refit
// Selection (Alg. 2 "best model", read as: most inliers, ties to the lowest
// index) is recomputed by every block from the counts; then the FP64 moments
// (n, sum q, sum q q^T with q = p - p0 of j*) of j*'s inliers are summed per
// fixed chunk of the point list, in a fixed order.
constexpr int kChunkSteps = kRefitChunk / kBlock;  // points per thread of a refit / removal chunk

// Symmetric 3x3 eigenproblem by cyclic Jacobi rotations in the tau form
// (a'_rp = a_rp - s (a_rq + tau a_rp), tau = s / (1 + c)); columns of v are
// the eigenvectors.
__device__ void jacobi3(double a[3][3], double v[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) v[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off == 0.0 || off <= 1e-40 * dia) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = a[p][q];
                if (apq == 0.0) continue;
                const double theta = 0.5 * (a[q][q] - a[p][p]) / apq;
                double t = 1.0 / (fabs(theta) + sqrt(1.0 + theta * theta));
                if (theta < 0.0) t = -t;
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c, tau = s / (1.0 + c);
                a[p][p] -= t * apq;
                a[q][q] += t * apq;
                a[p][q] = a[q][p] = 0.0;
                const int o = 3 - p - q;  // the remaining index
                const double g = a[o][p], hh = a[o][q];
                a[o][p] = a[p][o] = g - s * (hh + g * tau);
                a[o][q] = a[q][o] = hh + s * (g - hh * tau);
                for (int k = 0; k < 3; ++k) {
                    const double vg = v[k][p], vh = v[k][q];
                    v[k][p] = vg - s * (vh + vg * tau);
                    v[k][q] = vh + s * (vg - vh * tau);
                }
            }
    }
}

// The longest of the three pairwise cross products of the rows of A - l I
// (for l an eigenvalue, the rows span a plane whose normal is its
// eigenvector); returns its squared length.
__device__ __forceinline__ double row_cross(const double a[3][3], double l, double n[3]) {
    const double r[3][3] = {{a[0][0] - l, a[0][1], a[0][2]}, {a[0][1], a[1][1] - l, a[1][2]},
                            {a[0][2], a[1][2], a[2][2] - l}};
    const int pu[3] = {0, 0, 1}, pw[3] = {1, 2, 2};
    double best = -1.0;
    for (int k = 0; k < 3; ++k) {
        const double* u = r[pu[k]];
        const double* w = r[pw[k]];
        const double x = u[1] * w[2] - u[2] * w[1];
        const double y = u[2] * w[0] - u[0] * w[2];
        const double z = u[0] * w[1] - u[1] * w[0];
        const double q = x * x + y * y + z * z;
        if (q > best) {
            best = q;
            n[0] = x; n[1] = y; n[2] = z;
        }
    }
    return best;
}

// Eigenvector of the smallest eigenvalue l3 of a symmetric positive
// semi-definite 3x3 matrix A (a scatter matrix), unnormalised.  l3 is first
// approached as the smallest root of det(A - l I) = -l^3 + t2 l^2 - t1 l + t0
// (t2 = trace, t1 = sum of the principal 2x2 minors, t0 = det A): on [0, l3]
// that cubic decreases and is convex, so Newton steps from l = 0 climb to l3
// from below without overshoot; they stop when a step no longer increases l.
// t0 cancels badly when l3 is small, so the eigenvector from the rows of
// A - l I (row_cross) is refined twice by the Rayleigh quotient l = n.A n /
// n.n, whose error is quadratic in the eigenvector's; the result is as
// accurate as a backward-stable solver's (about u l1 / (l2 - l3)).  A
// handful of FP64 divisions instead of the dozens of rotations of Jacobi's
// method.  Returns false when l3 is not separated from l2 (the longest cross
// product is negligible), leaving the case to Jacobi.
__device__ bool smallest_eigvec(const double a[3][3], double n[3]) {
    const double t2 = a[0][0] + a[1][1] + a[2][2];
    const double c00 = a[1][1] * a[2][2] - a[1][2] * a[1][2];
    const double c01 = a[0][2] * a[1][2] - a[0][1] * a[2][2];
    const double c02 = a[0][1] * a[1][2] - a[1][1] * a[0][2];
    const double t1 = c00 + (a[0][0] * a[2][2] - a[0][2] * a[0][2]) + (a[0][0] * a[1][1] - a[0][1] * a[0][1]);
    const double t0 = a[0][0] * c00 + a[0][1] * c01 + a[0][2] * c02;
    double l = 0.0;
    for (int it = 0; it < 32; ++it) {
        const double p = ((t2 - l) * l - t1) * l + t0;
        const double dp = (2.0 * t2 - 3.0 * l) * l - t1;
        if (!(dp < 0.0)) break;
        const double ln = l - p / dp;
        if (!(ln > l)) break;
        l = ln;
    }
    double best = row_cross(a, l, n);
    for (int pass = 0; pass < 2; ++pass) {
        const double x = n[0], y = n[1], z = n[2];
        const double ax = a[0][0] * x + a[0][1] * y + a[0][2] * z;
        const double ay = a[0][1] * x + a[1][1] * y + a[1][2] * z;
        const double az = a[0][2] * x + a[1][2] * y + a[2][2] * z;
        l = (x * ax + y * ay + z * az) / (x * x + y * y + z * z);
        best = row_cross(a, l, n);
    }
    // |cross| ~ l1 (l2 - l3): a gap below 1e-12 of the trace goes to Jacobi
    const double g = 1e-24 * t2 * t2 * t2 * t2;
    return best > g && best < INFINITY;
}

// Reduce the chunk moments in a fixed order (thread t sums chunks t, t+256,
// ... in order, then a butterfly over each wave's lanes and the four waves in
// order), so every block obtains the same bits.  Then the least-squares plane: centroid c = shift + S/n,
// scatter C = Q - S S^T / n, normal = eigenvector of the smallest eigenvalue,
// d = -n.c, flipped so that d >= 0.  All threads call; thread 0 solves.
__device__ void solve_refit(const FrameDev& f, int M, double sx, double sy, double sz, double* plane, double* centroid,
                            double* nmom, double* sh) {
    const int nch = (M + kRefitChunk - 1) / kRefitChunk;
    const gf64_cptr part = (gf64_cptr)f.partials;
    double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = threadIdx.x; c < nch; c += kBlock)
#pragma unroll
        for (int k = 0; k < 10; ++k) m[k] += part[(size_t)c * 10 + k];
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = wave_sum_d(m[k]);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 10; ++k) sh[(threadIdx.x >> 6) * 10 + k] = m[k];
    __syncthreads();
    if (threadIdx.x != 0) return;
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = ((sh[k] + sh[10 + k]) + sh[20 + k]) + sh[30 + k];
    const double n = m[0];
    const double mx = m[1] / n, my = m[2] / n, mz = m[3] / n;
    double a[3][3];
    a[0][0] = m[4] - m[1] * mx; a[0][1] = m[5] - m[1] * my; a[0][2] = m[6] - m[1] * mz;
    a[1][1] = m[7] - m[2] * my; a[1][2] = m[8] - m[2] * mz; a[2][2] = m[9] - m[3] * mz;
    a[1][0] = a[0][1]; a[2][0] = a[0][2]; a[2][1] = a[1][2];
    double nv[3];
    if (!smallest_eigvec(a, nv)) {
        double v[3][3];
        jacobi3(a, v);
        int kmin = 0;
        if (a[1][1] < a[kmin][kmin]) kmin = 1;
        if (a[2][2] < a[kmin][kmin]) kmin = 2;
        nv[0] = v[0][kmin]; nv[1] = v[1][kmin]; nv[2] = v[2][kmin];
    }
    double nx = nv[0], ny = nv[1], nz = nv[2];
    const double nn = sqrt(nx * nx + ny * ny + nz * nz);
    nx /= nn; ny /= nn; nz /= nn;
    const double cx = sx + mx, cy = sy + my, cz = sz + mz;
    double d = -(nx * cx + ny * cy + nz * cz);
    if (d < 0.0) {
        nx = -nx; ny = -ny; nz = -nz; d = -d;
    }
    plane[0] = nx; plane[1] = ny; plane[2] = nz; plane[3] = d;
    centroid[0] = cx; centroid[1] = cy; centroid[2] = cz;
    *nmom = n;
}

// The tiles that a wave takes in chunk c of a refit or removal pass (step s:
// tile (c chunk + s 256) / 64 + wave) which hold no point with |n.p + d| < t
// for the plane h, decided from the tile boxes as the scorer decides them
// (hi = t + 16 u (P1 + |d|)): bit s, the same in every lane.  Tiles of padding
// only and tiles past the chunk's end e are in the set too.  Lane s gets the
// number of points of step s's tile in *cnt (0 in other lanes).
__device__ __forceinline__ unsigned long long tiles_outside(const FrameDev& f, int c, int e, float4 h, float hi,
                                                            int* cnt) {
    const int lane = threadIdx.x & 63;
    const int first = c * kRefitChunk + lane * kBlock + (threadIdx.x & ~63);  // the tile's first point (lane < steps)
    bool out = true;
    *cnt = 0;
    if (lane < kChunkSteps && first < e) {
        const float4 bc = ld_global4(f.tbox, 2 * (first >> 6));
        const float4 be = ld_global4(f.tbox, 2 * (first >> 6) + 1);
        *cnt = __float_as_int(bc.w);
        const float a = fabsf(fmaf(h.x, bc.x, fmaf(h.y, bc.y, fmaf(h.z, bc.z, h.w))));
        const float ext = fmaf(fabsf(h.x), be.x, fmaf(fabsf(h.y), be.y, fabsf(h.z) * be.z));
        out = *cnt == 0 || a - ext >= hi;
    }
    return __ballot(out);
}

__global__ __launch_bounds__(kBlock) void k_refit_moments(const FrameDev* __restrict__ tab, int r) {
    __shared__ int shk[8];
    __shared__ double shd[4][10];
    const FrameDev& f = tab[blockIdx.z];
    RoundState* st = f.st;
    const RoundRec rr = round_rec(f, r);
    if (!rr.active) return;
    const int M = rr.Mlen;
    const int nch = (M + kRefitChunk - 1) / kRefitChunk;
    if ((int)blockIdx.x >= nch) return;
    if (blockIdx.x == 0 && f.dbg.counts)
        for (int j = threadIdx.x; j < f.hyps; j += kBlock) f.dbg.counts[(size_t)r * f.hyps + j] = f.counts[j];
    const int js = select_jstar(f, shk);
    if (js < 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->round[r].stop = 1;
            if (f.dbg.round_info) {
                int32_t* ri = f.dbg.round_info + 4 * r;
                ri[0] = -1; ri[1] = 0; ri[2] = 0; ri[3] = 1;
            }
        }
        return;
    }
    const float4 h = ld_global4(f.hyp, js);
    const float4 p0 = ld_global4(f.hyp_p0, js);  // the first point of j*'s triple
    const double sx = p0.x, sy = p0.y, sz = p0.z;
    const float t = f.thresh;
    const float hi = t + 16.f * 5.9604645e-8f * (__uint_as_float(f.st->p1max_bits) + fabsf(h.w));
    const float4* __restrict__ pts = f.list[r & 1];
    for (int c = blockIdx.x; c < nch; c += gridDim.x) {
        double m[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        const int e = min(M, (c + 1) * kRefitChunk);
        // tiles without inliers add nothing: their points are not loaded
        int tcnt;
        const unsigned long long skip = tiles_outside(f, c, e, h, hi, &tcnt);
        // every other point of this thread in flight at once, then accumulated in index order
        float4 pp[kChunkSteps];
#pragma unroll
        for (int s = 0; s < kChunkSteps; ++s)
            pp[s] = (skip >> s) & 1ull ? pad_point() : ld_global4(pts, min(c * kRefitChunk + s * kBlock + (int)threadIdx.x, e - 1));
#pragma unroll
        for (int s = 0; s < kChunkSteps; ++s) {
            const float4 p = pp[s];
            if (!(c * kRefitChunk + s * kBlock + (int)threadIdx.x < e && fabsf(canon_res(h, p.x, p.y, p.z)) < t)) continue;
            const double qx = (double)p.x - sx, qy = (double)p.y - sy, qz = (double)p.z - sz;
            m[0] += 1.0;
            m[1] += qx; m[2] += qy; m[3] += qz;
            m[4] += qx * qx; m[5] += qx * qy; m[6] += qx * qz;
            m[7] += qy * qy; m[8] += qy * qz; m[9] += qz * qz;
            if (f.dbg.masks) {
                const int off = f.L[__float_as_int(p.w)];
                const int y = off / f.pitch, x = off - y * f.pitch;
                f.dbg.masks[(size_t)r * f.W * f.H + (size_t)y * f.W + x] |= 1;
            }
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) m[k] = wave_sum_d(m[k]);
        __syncthreads();
        if ((threadIdx.x & 63) == 0)
            for (int k = 0; k < 10; ++k) shd[threadIdx.x >> 6][k] = m[k];
        __syncthreads();
        if (threadIdx.x < 10) {
            const int k = threadIdx.x;
            f.partials[(size_t)c * 10 + k] = ((shd[0][k] + shd[1][k]) + shd[2][k]) + shd[3][k];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->round[r].stop = 0;
        st->round[r].jstar = js;
    }
}

// ------------------------------------------------------------------ removal
// |F| per chunk for the removal, F = the refit plane's inliers, and the
// padded length of the chunk's run of survivors in the next round's list.
// Every block first solves the refit plane itself (solve_refit: the same
// reduction order in every block, so the same plane bit for bit) while the
// points of its first chunk are already on their way; block 0 stores the
// plane, the centroid and |S|.  The grid gives each frame only a few blocks
// per CU, so the redundant solves run side by side, once per block.
__global__ __launch_bounds__(kBlock) void k_refit_final(const FrameDev* __restrict__ tab, int r) {
    __shared__ int sh[8];
    __shared__ double s_plane[4], s_cent[3], s_n;
    __shared__ double s_red[4 * 10];
    const FrameDev& f = tab[blockIdx.z];
    const RoundRec rr = round_rec(f, r);
    if (!rr.active || rr.stop) return;
    const int M = rr.Mlen;
    const int nch = (M + kRefitChunk - 1) / kRefitChunk;
    if ((int)blockIdx.x >= nch) return;
    const float t = f.thresh;
    const float4* __restrict__ pts = f.list[r & 1];
    int c = blockIdx.x;
    float4 pp[kChunkSteps];
    int e = min(M, (c + 1) * kRefitChunk);
#pragma unroll
    for (int s = 0; s < kChunkSteps; ++s) pp[s] = ld_global4(pts, min(c * kRefitChunk + s * kBlock + (int)threadIdx.x, e - 1));
    const float4 p0 = ld_global4(f.hyp_p0, rr.jstar);  // the moments' origin
    solve_refit(f, M, p0.x, p0.y, p0.z, s_plane, s_cent, &s_n, s_red);
    __syncthreads();
    const SplitPlane q = split_plane(s_plane);
    // the refit plane rounded to FP32 differs from it by at most u/2 (|p|_1 + |d|) in a
    // residual, which the box test's margin covers along with refit_res's own error
    const float4 qf = make_float4(q.hx, q.hy, q.hz, q.hd);
    const float hi = t + 16.f * 5.9604645e-8f * (__uint_as_float(f.st->p1max_bits) + fabsf(q.hd));
    int keep_skipped = 0;  // points of this lane's skipped tile (lanes below the step count)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        RoundState* st = f.st;
        for (int k = 0; k < 4; ++k) st->plane[k] = s_plane[k];
        for (int k = 0; k < 3; ++k) st->centroid[k] = s_cent[k];
        st->s_count = (int)s_n;
    }
    while (true) {
        int nF = 0, keep = 0;
#pragma unroll
        for (int s = 0; s < kChunkSteps; ++s) {
            const bool in = c * kRefitChunk + s * kBlock + (int)threadIdx.x < e;
            const bool f_in = in && fabsf(refit_res(q, pp[s].x, pp[s].y, pp[s].z)) < t;  // padding (NaN) never is
            nF += f_in ? 1 : 0;
            keep += (in && !f_in && pp[s].x == pp[s].x) ? 1 : 0;
        }
        keep += keep_skipped;
        block_sum2(nF, keep, sh);
        if (threadIdx.x == 0) {
            f.chunk_cnt[c] = nF;
            f.chunk_run[c] = align64(keep);
        }
        c += gridDim.x;
        if (c >= nch) break;
        e = min(M, (c + 1) * kRefitChunk);
        // later chunks: a tile that the boxes put wholly outside the refit plane's band
        // keeps all its points, which are then not loaded
        int tcnt;
        const unsigned long long skip = tiles_outside(f, c, e, qf, hi, &tcnt);
        keep_skipped = ((skip >> (threadIdx.x & 63)) & 1ull) ? tcnt : 0;
#pragma unroll
        for (int s = 0; s < kChunkSteps; ++s)
            pp[s] = (skip >> s) & 1ull ? pad_point() : ld_global4(pts, min(c * kRefitChunk + s * kBlock + (int)threadIdx.x, e - 1));
    }
}

// F = the refit plane's inliers among R_r (reading R18 of Alg. 2's model
// update).  If |F| >= min_inliers: label F with r, mark it assigned, write
// the plane record, and write each chunk's survivors, in order, as one run
// padded to a multiple of 64 into the next round's list (at the sum of the
// earlier chunks' runs), assembled in LDS and stored coalesced, then the
// bounding boxes of the run's tiles from the LDS copy; otherwise the frame
// stops without emitting.
__global__ __launch_bounds__(kBlock) void k_apply(const FrameDev* __restrict__ tab, int r) {
    __shared__ int sh[8];
    __shared__ int s_cnt[kChunkSteps][kBlock / 64];
    __shared__ float4 s_run[kRefitChunk];  // the chunk's run of survivors and padding
    const FrameDev& f = tab[blockIdx.z];
    RoundState* st = f.st;
    const RoundRec rr = round_rec(f, r);
    if (!rr.active || rr.stop) return;
    const int M = rr.Mlen;
    const int nch = (M + kRefitChunk - 1) / kRefitChunk;
    // a block takes a contiguous run of chunks, whose runs of survivors follow each other
    const int per = (nch + (int)gridDim.x - 1) / (int)gridDim.x;
    const int c0 = (int)blockIdx.x * per, c1 = min(nch, c0 + per);
    if (c0 >= nch) return;
    // |F| and the runs of the chunks before this block's first one, in one pass
    const gi32_cptr ccnt = (gi32_cptr)f.chunk_cnt;
    const gi32_cptr crun = (gi32_cptr)f.chunk_run;
    int ftot = 0, pre = 0;
    for (int c = threadIdx.x; c < nch; c += kBlock) {
        ftot += ccnt[c];
        pre += c < c0 ? crun[c] : 0;
    }
    block_sum2(ftot, pre, sh);
    const bool emit = ftot >= f.min_inliers;
    if (blockIdx.x == 0) {
        int rtot = 0;
        for (int c = threadIdx.x; c < nch; c += kBlock) rtot += crun[c];
        rtot = block_sum(rtot, sh);
        if (threadIdx.x == 0) {
            const int next = rr.M - (emit ? ftot : 0);
            if (emit) {
                pp_plane pl;
                for (int k = 0; k < 3; ++k) pl.n[k] = st->plane[k];
                pl.d = st->plane[3];
                for (int k = 0; k < 3; ++k) pl.centroid[k] = st->centroid[k];
                pl.inliers = ftot;
                pl.hyp_index = rr.jstar;
                f.planes[r] = pl;
                f.n_planes[0] = r + 1;
            }
            st->round[r + 1].M = next;
            st->round[r + 1].Mlen = rtot;
            st->round[r + 1].active = (emit && next >= 3 && r + 1 < f.max_planes) ? 1 : 0;
            if (f.dbg.round_info) {
                int32_t* ri = f.dbg.round_info + 4 * r;
                ri[0] = rr.jstar; ri[1] = st->s_count; ri[2] = ftot; ri[3] = emit ? 0 : 2;
            }
        }
    }
    if (!emit) return;
    const SplitPlane q = split_plane(st->plane);
    const float t = f.thresh;
    const float4* __restrict__ pts = f.list[r & 1];
    float4* __restrict__ out = f.list[(r + 1) & 1];
    const gi32_cptr Lg = (gi32_cptr)f.L;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = c0; c < c1; ++c) {
        const int start = pre;
        const int e = min(M, (c + 1) * kRefitChunk);
        // every point of this thread in flight at once: point c*chunk + s*256 + tid of step s
        float4 p[kChunkSteps];
#pragma unroll
        for (int s = 0; s < kChunkSteps; ++s) p[s] = ld_global4(pts, min(c * kRefitChunk + s * kBlock + (int)threadIdx.x, e - 1));
        bool inF[kChunkSteps];
        unsigned long long keepm[kChunkSteps];
#pragma unroll
        for (int s = 0; s < kChunkSteps; ++s) {
            const bool in = c * kRefitChunk + s * kBlock + (int)threadIdx.x < e;
            inF[s] = in && fabsf(refit_res(q, p[s].x, p[s].y, p[s].z)) < t;
            keepm[s] = __ballot(in && !inF[s] && p[s].x == p[s].x);
            if (lane == 0) s_cnt[s][wave] = __popcll(keepm[s]);
        }
        // the pixels of the inliers, all looked up before any store
        int off[kChunkSteps];
#pragma unroll
        for (int s = 0; s < kChunkSteps; ++s) off[s] = Lg[inF[s] ? __float_as_int(p[s].w) : 0];
#pragma unroll
        for (int s = 0; s < kChunkSteps; ++s)
            if (inF[s]) {
                f.labels[off[s]] = (int8_t)r;
                f.taken[__float_as_int(p[s].w)] = 1;
                if (f.dbg.masks) {
                    const int y = off[s] / f.pitch, x = off[s] - y * f.pitch;
                    f.dbg.masks[(size_t)r * f.W * f.H + (size_t)y * f.W + x] |= 2;
                }
            }
        __syncthreads();  // s_cnt
        // survivors keep their order: step-major, then wave, then lane; then the padding
        int base = start;
#pragma unroll
        for (int s = 0; s < kChunkSteps; ++s) {
            int mine = base;
            for (int w = 0; w < kBlock / 64; ++w) {
                const int n = s_cnt[s][w];
                mine += w < wave ? n : 0;
                base += n;
            }
            if ((keepm[s] >> lane) & 1ull) s_run[mine - start + __popcll(keepm[s] & lanemask_lt())] = p[s];
        }
        const int end = align64(base);
        for (int i = base + (int)threadIdx.x; i < end; i += kBlock) s_run[i - start] = pad_point();
        __syncthreads();  // the run is in LDS for the whole block
        // stored in order, one 16-byte store per thread and step; the tile boxes from the LDS copy
        for (int i = threadIdx.x; i < end - start; i += kBlock) out[start + i] = s_run[i];
        tile_boxes(s_run, (end - start) >> 6, f.tbox + 2 * (start >> 6), wave, kBlock / 64);
        pre = end;  // the next chunk's run follows this one's
        __syncthreads();  // s_cnt and s_run are reused by the next chunk
    }
}

// ------------------------------------------------------------------ launchers
static const int kHB[kNumHB] = {8, 16, 32, 64, 128, 256};  // 64 Q: the tile-culled scorer, Q per lane
static const int kChunk[kNumChunk] = {1024, 2048, 4096, 8192};

int hb_value(int i) { return kHB[i]; }
int chunk_value(int i) { return kChunk[i]; }
bool t_supported(int t) { return t == 1 || t == 2 || t == 3 || t == 4 || t == 5 || t == 8 || t == 10; }

template <int TX, int TY, int T>
static void diffuse_pass(const FrameDev* tab, int nf, int maxW, int maxH, int it, int first, int last, int src,
                         int dst, hipStream_t s) {
    dim3 grid((maxW + TX - 1) / TX, (maxH + TY - 1) / TY, nf);
    hipLaunchKernelGGL((k_diffuse<TX, TY, T>), grid, dim3(kBlock), 0, s, tab, it, first, last, src, dst);
}

// Register-resident form: 4 waves of 64 lanes side by side, each writing
// 64 - 2T columns and TY rows.
template <int TY, int T>
static void diffuse_pass_wc(const FrameDev* tab, int nf, int maxW, int maxH, int it, int first, int last, int src,
                            int dst, hipStream_t s) {
    constexpr int OW = 64 - 2 * T;
    dim3 grid((maxW + (kBlock / 64) * OW - 1) / ((kBlock / 64) * OW), (maxH + TY - 1) / TY, nf);
    hipLaunchKernelGGL((k_diffuse_wc<TY, T>), grid, dim3(kBlock), 0, s, tab, it, first, last, src, dst);
}

template <int TY>
static void diffuse_pass_wc_t(int T, const FrameDev* tab, int nf, int maxW, int maxH, int it, int first, int last,
                              int src, int dst, hipStream_t s) {
    switch (T) {
        case 1: diffuse_pass_wc<TY, 1>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        case 2: diffuse_pass_wc<TY, 2>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        case 3: diffuse_pass_wc<TY, 3>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        case 4: diffuse_pass_wc<TY, 4>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        case 5: diffuse_pass_wc<TY, 5>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        case 8: diffuse_pass_wc<TY, 8>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        default: diffuse_pass_wc<TY, 10>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
    }
}

template <int TX, int TY>
static void diffuse_pass_t(int T, const FrameDev* tab, int nf, int maxW, int maxH, int it, int first, int last,
                           int src, int dst, hipStream_t s) {
    switch (T) {
        case 1: diffuse_pass<TX, TY, 1>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        case 2: diffuse_pass<TX, TY, 2>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        case 3: diffuse_pass<TX, TY, 3>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        case 4: diffuse_pass<TX, TY, 4>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        case 5: diffuse_pass<TX, TY, 5>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        case 8: diffuse_pass<TX, TY, 8>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        default: diffuse_pass<TX, TY, 10>(tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
    }
}

// All frames of a table run max(iters) iterations in passes of T, with one
// discretisation; frames with other iteration counts or schemes must not be
// mixed with them (the batch path groups frames by both).
hipError_t launch_diffuse(const FrameDev* tab, int nf, int maxW, int maxH, int iters, int scheme, const Tuning& tu,
                          hipStream_t s) {
    if (iters <= 0) {
        hipLaunchKernelGGL(k_diffuse_copy, dim3((maxW + 63) / 64, (maxH + 3) / 4, nf), dim3(kBlock), 0, s, tab);
        return hipGetLastError();
    }
    if (scheme != PP_DIFFUSE_EDGE4) {
        const dim3 grid((maxW + kVarTX - 1) / kVarTX, (maxH + kVarTY - 1) / kVarTY, nf);
        for (int done = 0, src = 0; done < iters; src ^= 1) {
            const int it = iters - done < kVarT ? iters - done : kVarT;
            const int first = done == 0, last = done + it == iters;
            if (scheme == PP_DIFFUSE_PIXEL)
                hipLaunchKernelGGL(k_diffuse_var<PP_DIFFUSE_PIXEL>, grid, dim3(kBlock), 0, s, tab, it, first, last, src,
                                   src ^ 1);
            else
                hipLaunchKernelGGL(k_diffuse_var<PP_DIFFUSE_EDGE8>, grid, dim3(kBlock), 0, s, tab, it, first, last, src,
                                   src ^ 1);
            done += it;
        }
        return hipGetLastError();
    }
    const int T = tu.diffuse_t;
    int done = 0, src = 0, pass = 0;
    while (done < iters) {
        const int it = iters - done < T ? iters - done : T;
        const int first = done == 0, last = done + it == iters;
        const int dst = src ^ 1;
        switch (tu.diffuse_tile) {
            case 0: diffuse_pass_t<64, 16>(T, tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
            case 1: diffuse_pass_t<128, 16>(T, tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
            case 2: diffuse_pass_t<64, 32>(T, tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
            case 3: diffuse_pass_t<128, 32>(T, tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
            case 4: diffuse_pass_wc_t<8>(T, tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
            default: diffuse_pass_wc_t<16>(T, tab, nf, maxW, maxH, it, first, last, src, dst, s); break;
        }
        done += it;
        src = dst;
        ++pass;
    }
    return hipGetLastError();
}

hipError_t launch_normals(const FrameDev* tab, int nf, int max_px, bool count, hipStream_t s) {
    const int nch = (max_px + kValidChunk - 1) / kValidChunk;
    hipLaunchKernelGGL(k_normals, dim3(nch > 0 ? nch : 1, 1, nf), dim3(kBlock), 0, s, tab, count ? 1 : 0);
    return hipGetLastError();
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Blocks per frame for a pass over nch chunks: one per chunk up to cap blocks over all nf
// frames, then fewer blocks that take several chunks each.  A capped count is made odd:
// workgroups go to the 8 XCDs in turn, and with a multiple of 8 blocks a frame, block x of
// every frame would land on the same XCD.
static int pass_blocks(int nch, int nf, int cap) {
    const int per = std::max(cap / std::max(nf, 1), 1);
    if (nch <= per) return clampi(nch, 1, 1024);
    return clampi(per | 1, 1, 1023);
}

// Blocks of the moments, removal and valid-list passes over all frames (32 per CU).
constexpr int kPassBlocks = 8192;

hipError_t launch_valid_list(const FrameDev* tab, int nf, int max_px, int maxW, int maxH, bool counted, hipStream_t s) {
    const int nch = (max_px + kValidChunk - 1) / kValidChunk;
    const int gx = clampi(nch, 1, 1024);
    if (!counted) hipLaunchKernelGGL(k_valid_count, dim3(gx, 1, nf), dim3(kBlock), 0, s, tab);
    hipLaunchKernelGGL(k_valid_scatter, dim3(pass_blocks(nch, nf, kPassBlocks), 1, nf), dim3(kBlock), 0, s, tab);
    // block-order chunks: a frame's padded scan covers at most 3.4 W H + 70
    // positions, and at most the padded maxW x maxH grid; one block per chunk
    const int64_t pad = kScanBlock;
    const int64_t grid = (maxW + pad - 1) / pad * pad * ((maxH + pad - 1) / pad * pad);
    const int64_t scan = grid < (int64_t)4 * max_px + 4096 ? grid : (int64_t)4 * max_px + 4096;
    const int gq = clampi((int)((scan + kValidChunk - 1) / kValidChunk), 1, 1024);
    hipLaunchKernelGGL(k_list0, dim3(gq, 1, nf), dim3(kBlock), 0, s, tab);
    return hipGetLastError();
}

template <int HB>
static void score_launch(const FrameDev* tab, int nf, int r, int max_pts, int max_hyps, int target,
                         hipStream_t s) {
    const int groups = (max_hyps + HB - 1) / HB;
    const int per_frame_cap = clampi(16384 / (nf > 0 ? nf : 1), 8, 4096);
    const int bx = clampi((max_pts + target - 1) / target, 1, clampi(per_frame_cap / groups, 1, 1024));
    hipLaunchKernelGGL((k_score<HB>), dim3(bx, groups, nf), dim3(kBlock), 0, s, tab, r);
}

// Tile-culled scoring (k_score_tiles), 64 Q hypotheses per block; the tile
// boxes are made at the round's start.
template <int PREC>
static void score_tiles_launch(const FrameDev* tab, int nf, int r, int max_pts, int max_hyps, int target, int q,
                               hipStream_t s) {
    const int groups = (max_hyps + 64 * q - 1) / (64 * q);
    const int per_frame_cap = clampi(16384 / (nf > 0 ? nf : 1), 8, 4096);
    const int bx = clampi((max_pts + target - 1) / target, 1, clampi(per_frame_cap / groups, 1, 1024));
    const dim3 grid(bx, groups, nf);
    if (q == 1) hipLaunchKernelGGL((k_score_tiles<PREC, 1>), grid, dim3(kBlock), 0, s, tab, r);
    else if (q == 2) hipLaunchKernelGGL((k_score_tiles<PREC, 2>), grid, dim3(kBlock), 0, s, tab, r);
    else hipLaunchKernelGGL((k_score_tiles<PREC, 4>), grid, dim3(kBlock), 0, s, tab, r);
}

// Tile-box culling: every matrix-core form, and the FP32 form at the culled tunings.
static bool culled(int precision, const Tuning& tu) { return precision != PP_SCORE_FP32 || tu.score_hb >= 3; }
static int tiles_q(const Tuning& tu) { return tu.score_hb <= 3 ? 1 : (tu.score_hb == 4 ? 2 : 4); }

static void score_dispatch(const FrameDev* tab, int nf, int r, int max_pts, int max_hyps, int precision,
                           const Tuning& tu, hipStream_t s) {
    const int target = chunk_value(tu.score_chunk);
    if (!culled(precision, tu)) {
        switch (tu.score_hb) {
            case 0: score_launch<8>(tab, nf, r, max_pts, max_hyps, target, s); break;
            case 1: score_launch<16>(tab, nf, r, max_pts, max_hyps, target, s); break;
            default: score_launch<32>(tab, nf, r, max_pts, max_hyps, target, s); break;
        }
        return;
    }
    const int q = tiles_q(tu);
    switch (precision) {
        case PP_SCORE_MFMA_F32: score_tiles_launch<PP_SCORE_MFMA_F32>(tab, nf, r, max_pts, max_hyps, target, q, s); break;
        case PP_SCORE_BF16: score_tiles_launch<PP_SCORE_BF16>(tab, nf, r, max_pts, max_hyps, target, q, s); break;
        case PP_SCORE_FP16: score_tiles_launch<PP_SCORE_FP16>(tab, nf, r, max_pts, max_hyps, target, q, s); break;
        default: score_tiles_launch<PP_SCORE_FP32>(tab, nf, r, max_pts, max_hyps, target, q, s); break;
    }
}

// Blocks of the final pass over all frames (8 per CU): more would repeat the
// plane solve in more block waves.
constexpr int kFinalBlocks = 2048;


// One RANSAC round for every frame of the table: hypotheses, scoring,
// selection and moments, the refit plane and its inliers per chunk, the
// removal with the next round's list and tile boxes.
hipError_t launch_round(const FrameDev* tab, int nf, int r, int max_px, int max_hyps, int precision,
                        const Tuning& tu, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const int bpf = (max_hyps + kHypPerBlock - 1) / kHypPerBlock;
    const int hyp_blocks = (bpf * nf + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL(k_round_start, dim3(hyp_blocks), dim3(kBlock), 0, s, tab, r, bpf, nf);
    if (ev0) (void)hipEventRecord(ev0, s);
    const int max_pts = max_px;  // the longest list: the scan positions of the largest frame
    score_dispatch(tab, nf, r, max_pts, max_hyps, precision, tu, s);
    if (ev1) (void)hipEventRecord(ev1, s);
    // the final count solves the plane in every block, so it gets fewer blocks (in late rounds
    // only the first few chunks of a frame hold points, which the odd capped grids spread over
    // the XCDs)
    const int nch = (max_pts + kRefitChunk - 1) / kRefitChunk;
    const int gx = pass_blocks(nch, nf, kPassBlocks);
    hipLaunchKernelGGL(k_refit_moments, dim3(gx, 1, nf), dim3(kBlock), 0, s, tab, r);
    hipLaunchKernelGGL(k_refit_final, dim3(pass_blocks(nch, nf, kFinalBlocks), 1, nf), dim3(kBlock), 0, s, tab, r);
    hipLaunchKernelGGL(k_apply, dim3(gx, 1, nf), dim3(kBlock), 0, s, tab, r);
    return hipGetLastError();
}

hipError_t launch_hyp_from_triples(const FrameDev* tab, const int32_t* triples, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_hyp_from_triples, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, tab, triples, n);
    return hipGetLastError();
}

hipError_t launch_score_only(const FrameDev* tab, int max_px, int n, int precision, const Tuning& tu, hipStream_t s) {
    score_dispatch(tab, 1, 0, max_px, n, precision, tu, s);
    return hipGetLastError();
}

}  // namespace ppk
