// Region-mode RANSAC for gfx950: Alg. 2 as printed, for every region of a
// label image at once.
//
//   k_reg_count    points per (pixel block, region); labels cleared
//   k_reg_scan     region sizes, list offsets, scoring-chunk offsets
//   k_reg_scatter  each region's points in row-major order (ordered, stable)
//   k_reg_hypgen   hypothesis j of region g: three distinct list positions
//                  from Philox4x64-10, counter (j, g, b, 1); FP32 plane
//   k_reg_score    per (region chunk, hypothesis): FP64 sum of |r| over the
//                  chunk in list order, and the inlier count (|r| < t)
//   k_reg_select   per region: errors summed over chunks in order; the first
//                  smallest error wins; stored iff 10 inliers > 9 n_g
//   k_reg_label    per chunk of a stored region: labels of the inliers and
//                  FP64 partial sums of their coordinates (fixed order)
//   k_reg_centroid per stored region: the partial sums in chunk order
//
// Every sum has a fixed order, so results do not depend on scheduling.  The
// residual is the canonical FP32 expression the whole-frame scorers use.

#include <math.h>

#include "pp_device.h"
#include "pp_internal.h"

namespace ppk {

namespace {

constexpr int kRegMax = kMaxRounds;  // regions per frame (labels are int8)

__device__ __forceinline__ float3 reg_point(const RegionDev& r, int off) {
    const size_t plane = (size_t)r.H * r.pitch;
    return make_float3(r.pts[off], r.pts[plane + off], r.pts[2 * plane + off]);
}

__device__ __forceinline__ int reg_of(const RegionDev& r, int off) {
    const int g = r.region[off];
    return (g >= 0 && g < r.R && (r.valid[off] & 1)) ? g : -1;
}

__global__ __launch_bounds__(kBlock) void k_reg_count(RegionDev r) {
    __shared__ int hist[kRegMax];
    for (int g = threadIdx.x; g < r.R; g += kBlock) hist[g] = 0;
    __syncthreads();
    const int npx = r.W * r.H;
    const int base = blockIdx.x * kRegionPxChunk;
    for (int i = threadIdx.x; i < kRegionPxChunk; i += kBlock) {
        const int p = base + i;
        if (p >= npx) break;
        const int y = p / r.W, x = p - y * r.W;
        const int off = y * r.pitch + x;
        r.labels[off] = -1;
        const int g = reg_of(r, off);
        if (g >= 0) atomicAdd(&hist[g], 1);
    }
    __syncthreads();
    for (int g = threadIdx.x; g < r.R; g += kBlock) r.bcnt[blockIdx.x * r.R + g] = hist[g];
}

// One block.  bcnt[b][g] becomes the list position of block b's first point of region g.
__global__ __launch_bounds__(kBlock) void k_reg_scan(RegionDev r) {
    __shared__ int n[kRegMax];
    __shared__ int off[kRegMax + 1];
    const int g = threadIdx.x;
    if (g < r.R) {
        int run = 0;
        for (int b = 0; b < r.nb; ++b) {
            const int c = r.bcnt[b * r.R + g];
            r.bcnt[b * r.R + g] = run;
            run += c;
        }
        n[g] = run;
        r.npts[g] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int o = 0, ch = 0;
        for (int k = 0; k < r.R; ++k) {
            off[k] = o;
            r.off[k] = o;
            r.choff[k] = ch;
            o += n[k];
            ch += (n[k] + kRegionChunk - 1) / kRegionChunk;
        }
        off[r.R] = o;
        r.off[r.R] = o;
        r.choff[r.R] = ch;
        *r.n_planes = 0;
    }
    __syncthreads();
    if (g < r.R)
        for (int b = 0; b < r.nb; ++b) r.bcnt[b * r.R + g] += off[g];
}

// Ordered scatter: the block walks its pixels 256 at a time; within a step a
// pixel's rank among equal labels comes from the waves before it and, inside
// its wave, from the lanes below it.
__global__ __launch_bounds__(kBlock) void k_reg_scatter(RegionDev r) {
    __shared__ int run[kRegMax];
    __shared__ int wc[kBlock / 64][kRegMax];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int g = threadIdx.x; g < r.R; g += kBlock) {
        run[g] = r.bcnt[blockIdx.x * r.R + g];
        for (int k = 0; k < kBlock / 64; ++k) wc[k][g] = 0;
    }
    __syncthreads();
    const int npx = r.W * r.H;
    const int base = blockIdx.x * kRegionPxChunk;
    for (int step = 0; step < kRegionPxChunk / kBlock; ++step) {
        const int p = base + step * kBlock + threadIdx.x;
        int off = 0, g = -1;
        if (p < npx) {
            const int y = p / r.W, x = p - y * r.W;
            off = y * r.pitch + x;
            g = reg_of(r, off);
        }
        unsigned long long pending = __ballot(g >= 0);
        int rank = 0;
        while (pending) {  // wave-uniform: one pass per distinct label in the wave
            const int leader = __ffsll(pending) - 1;
            const int L = __shfl(g, leader);
            const unsigned long long m = __ballot(g == L);
            if (g == L) rank = __popcll(m & lanemask_lt());
            if (lane == 0) wc[w][L] = __popcll(m);
            pending &= ~m;
        }
        __syncthreads();
        if (g >= 0) {
            int pos = run[g] + rank;
            for (int k = 0; k < w; ++k) pos += wc[k][g];
            r.list[pos] = off;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < r.R; k += kBlock) {
            int s = 0;
            for (int q = 0; q < kBlock / 64; ++q) {
                s += wc[q][k];
                wc[q][k] = 0;
            }
            run[k] += s;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_reg_hypgen(RegionDev r) {
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= r.R * r.hyps) return;
    const int g = idx / r.hyps, j = idx - g * r.hyps;
    const int n = r.npts[g];
    int slot[3] = {-1, -1, -1};
    int got = 0;
    for (int b = 0; b < 16 && got < 3 && n > 0; ++b) {
        uint64_t c[4] = {(uint64_t)j, (uint64_t)g, (uint64_t)b, 1ull};
        philox4x64_10(c, r.seed, r.frame_id);
        for (int q = 0; q < 4 && got < 3; ++q) {
            const int k = (int)__umul64hi(c[q], (uint64_t)n);
            bool dup = false;
            for (int s = 0; s < got; ++s) dup |= slot[s] == k;
            if (!dup) slot[got++] = k;
        }
    }
    float4 h = make_float4(0.f, 0.f, 0.f, __int_as_float(0x7fc00000));
    if (got == 3) {
        const int o = r.off[g];
        h = plane_from_points(reg_point(r, r.list[o + slot[0]]), reg_point(r, r.list[o + slot[1]]),
                              reg_point(r, r.list[o + slot[2]]));
    }
    for (int s = 0; s < 3; ++s) r.triples[3 * idx + s] = got == 3 ? slot[s] : -1;
    r.hyp[idx] = h;
    r.counts[idx] = 0;
}

// Block = one chunk of one region's list; its points are staged in LDS and
// every thread walks them in order for its hypotheses.
__global__ __launch_bounds__(kBlock) void k_reg_score(RegionDev r) {
    __shared__ float sx[kRegionChunk], sy[kRegionChunk], sz[kRegionChunk];
    const int c = blockIdx.x;
    if (c >= r.choff[r.R]) return;
    int lo = 0, hi = r.R - 1;  // the last region whose first chunk is <= c
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (r.choff[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    const int g = lo;
    const int k0 = r.off[g] + (c - r.choff[g]) * kRegionChunk;
    const int k1 = min(k0 + kRegionChunk, r.off[g + 1]);
    const int m = k1 - k0;
    for (int i = threadIdx.x; i < m; i += kBlock) {
        const float3 p = reg_point(r, r.list[k0 + i]);
        sx[i] = p.x;
        sy[i] = p.y;
        sz[i] = p.z;
    }
    __syncthreads();
    const float t = r.thresh;
    for (int j = threadIdx.x; j < r.hyps; j += kBlock) {
        const float4 h = r.hyp[g * r.hyps + j];
        double e = 0.0;
        int cnt = 0;
        if (h.w == h.w) {
            for (int i = 0; i < m; ++i) {
                const float a = fabsf(canon_res(h, sx[i], sy[i], sz[i]));
                e += (double)a;
                cnt += a < t;
            }
        }
        r.errp[(size_t)c * r.hyps + j] = e;
        if (cnt) atomicAdd(&r.counts[g * r.hyps + j], cnt);
    }
}

__global__ __launch_bounds__(kBlock) void k_reg_select(RegionDev r) {
    __shared__ double se[kBlock];
    __shared__ int sj[kBlock];
    const int g = blockIdx.x;
    const int c0 = r.choff[g], c1 = r.choff[g + 1];
    double best = __builtin_inf();
    int bj = -1;
    for (int j = threadIdx.x; j < r.hyps; j += kBlock) {
        const float4 h = r.hyp[g * r.hyps + j];
        double e = __builtin_inf();
        if (h.w == h.w) {
            e = 0.0;
            for (int c = c0; c < c1; ++c) e += r.errp[(size_t)c * r.hyps + j];
        }
        r.errors[g * r.hyps + j] = e;
        if (e < best) {
            best = e;
            bj = j;
        }
    }
    se[threadIdx.x] = best;
    sj[threadIdx.x] = bj;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double eo = se[threadIdx.x + s];
            const int jo = sj[threadIdx.x + s];
            const bool take = jo >= 0 && (sj[threadIdx.x] < 0 || eo < se[threadIdx.x] ||
                                          (eo == se[threadIdx.x] && jo < sj[threadIdx.x]));
            if (take) {
                se[threadIdx.x] = eo;
                sj[threadIdx.x] = jo;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int js = sj[0];
        const int n = r.npts[g];
        const int cnt = js >= 0 ? r.counts[g * r.hyps + js] : 0;
        const bool stored = js >= 0 && 10ll * cnt > 9ll * n;
        r.jstar[g] = js;
        pp_plane pl{};
        if (js >= 0) {
            const float4 h = r.hyp[g * r.hyps + js];
            pl.n[0] = h.x;
            pl.n[1] = h.y;
            pl.n[2] = h.z;
            pl.d = h.w;
        }
        pl.inliers = cnt;
        pl.hyp_index = stored ? js : -1;
        r.planes[g] = pl;
        if (stored) atomicAdd(r.n_planes, 1);
    }
}

// Labels and the centroid's partial sums, one block per 512-point chunk of a
// stored region's list: FP64 sums per thread in list order, then the waves
// in order, so the result does not depend on scheduling.
__global__ __launch_bounds__(kBlock) void k_reg_label(RegionDev r) {
    __shared__ double sh[3][kBlock / 64];
    const int c = blockIdx.x;
    if (c >= r.choff[r.R]) return;
    int lo = 0, hi = r.R - 1;  // the last region whose first chunk is <= c
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (r.choff[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    const int g = lo;
    const int js = r.jstar[g];
    if (js < 0 || r.planes[g].hyp_index < 0) return;
    const float4 h = r.hyp[g * r.hyps + js];
    const int k0 = r.off[g] + (c - r.choff[g]) * kRegionChunk;
    const int k1 = min(k0 + kRegionChunk, r.off[g + 1]);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int i = k0 + threadIdx.x; i < k1; i += kBlock) {
        const int off = r.list[i];
        const float3 p = reg_point(r, off);
        if (fabsf(canon_res(h, p.x, p.y, p.z)) < r.thresh) {
            r.labels[off] = (int8_t)g;
            s0 += p.x;
            s1 += p.y;
            s2 += p.z;
        }
    }
    s0 = wave_sum_d(s0);
    s1 = wave_sum_d(s1);
    s2 = wave_sum_d(s2);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = s0;
        sh[1][w] = s1;
        sh[2][w] = s2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) s += sh[threadIdx.x][k];
        r.cpart[(size_t)c * 3 + threadIdx.x] = s;
    }
}

// Centroid of each stored region: its chunks' partial sums in order.
__global__ __launch_bounds__(kBlock) void k_reg_centroid(RegionDev r) {
    const int g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= r.R || r.jstar[g] < 0 || r.planes[g].hyp_index < 0) return;
    double s[3] = {0.0, 0.0, 0.0};
    for (int c = r.choff[g]; c < r.choff[g + 1]; ++c)
        for (int a = 0; a < 3; ++a) s[a] += r.cpart[(size_t)c * 3 + a];
    const double cnt = (double)r.planes[g].inliers;
    for (int a = 0; a < 3; ++a) r.planes[g].centroid[a] = s[a] / cnt;
}

template <typename T>
T* carve(uintptr_t& p, size_t n) {
    T* q = reinterpret_cast<T*>(p);
    p += (n * sizeof(T) + 255) & ~size_t(255);
    return q;
}

}  // namespace

int region_blocks(int W, int H) { return (W * H + kRegionPxChunk - 1) / kRegionPxChunk; }

int region_max_chunks(int W, int H, int R) { return (W * H + kRegionChunk - 1) / kRegionChunk + R; }

size_t region_bind_scratch(RegionDev& r, void* scratch) {
    const uintptr_t base = reinterpret_cast<uintptr_t>(scratch);
    uintptr_t p = base;
    const size_t npx = (size_t)r.W * r.H, rh = (size_t)r.R * r.hyps;
    r.nb = region_blocks(r.W, r.H);
    r.bcnt = carve<int32_t>(p, (size_t)r.nb * r.R);
    r.off = carve<int32_t>(p, r.R + 1);
    r.choff = carve<int32_t>(p, r.R + 1);
    r.npts = carve<int32_t>(p, r.R);
    r.list = carve<int32_t>(p, npx);
    r.hyp = carve<float4>(p, rh);
    r.triples = carve<int32_t>(p, 3 * rh);
    r.errp = carve<double>(p, (size_t)region_max_chunks(r.W, r.H, r.R) * r.hyps);
    r.counts = carve<int32_t>(p, rh);
    r.errors = carve<double>(p, rh);
    r.jstar = carve<int32_t>(p, r.R);
    r.cpart = carve<double>(p, (size_t)region_max_chunks(r.W, r.H, r.R) * 3);
    return (size_t)(p - base);
}

size_t region_scratch_bytes(int W, int H, int R, int hyps) {
    RegionDev r{};
    r.W = W;
    r.H = H;
    r.R = R;
    r.hyps = hyps;
    return region_bind_scratch(r, nullptr);
}

hipError_t launch_regions(const RegionDev& r, hipStream_t s) {
    const dim3 blk(kBlock);
    hipLaunchKernelGGL(k_reg_count, dim3(r.nb), blk, 0, s, r);
    hipLaunchKernelGGL(k_reg_scan, dim3(1), blk, 0, s, r);
    hipLaunchKernelGGL(k_reg_scatter, dim3(r.nb), blk, 0, s, r);
    hipLaunchKernelGGL(k_reg_hypgen, dim3((r.R * r.hyps + kBlock - 1) / kBlock), blk, 0, s, r);
    hipLaunchKernelGGL(k_reg_score, dim3(region_max_chunks(r.W, r.H, r.R)), blk, 0, s, r);
    hipLaunchKernelGGL(k_reg_select, dim3(r.R), blk, 0, s, r);
    hipLaunchKernelGGL(k_reg_label, dim3(region_max_chunks(r.W, r.H, r.R)), blk, 0, s, r);
    hipLaunchKernelGGL(k_reg_centroid, dim3((r.R + kBlock - 1) / kBlock), blk, 0, s, r);
    return hipGetLastError();
}

}  // namespace ppk
