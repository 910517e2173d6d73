// Segmentation of the normal image for gfx950 (Sec. III-D: Canny edges on the
// normal image; the regions between the edges are the candidate planes that
// region-mode RANSAC fits).
//
//   k_seg_grad    Sobel sums of each normal channel (the kernels of Eq. 2),
//                 squared magnitude m2 = Exx + Eyy of the structure tensor,
//                 edge sector from (Exx - Eyy, 2 Exy); barrier where the 3x3
//                 window holds an invalid normal
//   k_seg_nms     non-maximum suppression along the sector, weak/strong by
//                 m2 > low^2 / m2 > high^2
//   k_uf_*        union-find on 8-connected edge pixels (hysteresis: a
//                 component is an edge iff it holds a strong pixel), then on
//                 4-connected region pixels (valid, no barrier, no edge pixel
//                 in the 3x3 window)
//   k_seg_cand/sort/label
//                 components of at least min_area pixels ranked by size, then
//                 smallest pixel index; at most max_regions get labels
//
// Every floating-point decision is the same FP32 expression, in the same
// order, as the CPU reference, so edges and regions are exact.  Union-find
// hooks the larger root under the smaller with compare-and-swap, so each
// component's root is its smallest pixel index whatever the schedule; no host
// synchronisation is needed.

#include <math.h>

#include "pp_device.h"
#include "pp_internal.h"

namespace ppk {

namespace {

constexpr uint8_t kBarrier = 4, kWeak = 8, kStrong = 16, kEdge = 32;

// Root of x, halving the path on the way: a non-root node is re-pointed to
// its grandparent, always an ancestor, so concurrent hooks of roots (the only
// other writes) stay valid; a node that is not a root never becomes one.
__device__ __forceinline__ int uf_find(int32_t* parent, int x) {
    while (true) {
        const int p = __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p == x) return x;
        const int gp = __hip_atomic_load(parent + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
}

__device__ __forceinline__ void uf_unite(int32_t* parent, int a, int b) {
    while (true) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicCAS(parent + a, a, b);
        if (old == a) return;
        a = old;
    }
}

__device__ __forceinline__ bool pix(const SegDev& s, int& x, int& y) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= s.W * s.H) return false;
    y = p / s.W;
    x = p - y * s.W;
    return true;
}

__global__ __launch_bounds__(kBlock) void k_seg_grad(SegDev s) {
    int x, y;
    if (blockIdx.x == 0 && threadIdx.x == 0) *s.ncand = 0;
    if (!pix(s, x, y)) return;
    const int p = y * s.W + x;
    s.strong[p] = 0;
    bool ok = x >= 1 && x < s.W - 1 && y >= 1 && y < s.H - 1;
    for (int dv = -1; dv <= 1 && ok; ++dv)
        for (int du = -1; du <= 1; ++du)
            if (!(s.valid[(y + dv) * s.pitch + x + du] & 2)) ok = false;
    if (!ok) {
        s.m2[p] = 0.f;
        s.meta[p] = kBarrier;
        return;
    }
    const size_t plane = (size_t)s.H * s.pitch;
    const int o = y * s.pitch + x;
    float exx = 0.f, eyy = 0.f, exy = 0.f;
    for (int c = 0; c < 3; ++c) {
        const float* ch = s.nrm + c * plane + o;
        const int P = s.pitch;
        const float gx = ((ch[-P + 1] - ch[-P - 1]) + 2.0f * (ch[1] - ch[-1])) + (ch[P + 1] - ch[P - 1]);
        const float gy = ((ch[P - 1] - ch[-P - 1]) + 2.0f * (ch[P] - ch[-P])) + (ch[P + 1] - ch[-P + 1]);
        exx = exx + gx * gx;
        eyy = eyy + gy * gy;
        exy = exy + gx * gy;
    }
    s.m2[p] = exx + eyy;
    const float A = exx - eyy, B = 2.0f * exy;
    uint8_t sec;
    if (fabsf(B) <= fabsf(A)) sec = A >= 0.f ? 0 : 2;
    else sec = B > 0.f ? 1 : 3;
    s.meta[p] = sec;
}

__global__ __launch_bounds__(kBlock) void k_seg_nms(SegDev s) {
    int x, y;
    if (!pix(s, x, y)) return;
    const int p = y * s.W + x;
    uint8_t m = s.meta[p];
    int cls = 0;
    if (!(m & kBarrier)) {
        const int sec = m & 3;
        const int du = sec == 2 ? 0 : 1, dv = sec == 0 ? 0 : (sec == 3 ? -1 : 1);
        const int xa = x + du, ya = y + dv, xb = x - du, yb = y - dv;
        const float ahead = (xa >= 0 && xa < s.W && ya >= 0 && ya < s.H) ? s.m2[ya * s.W + xa] : 0.f;
        const float behind = (xb >= 0 && xb < s.W && yb >= 0 && yb < s.H) ? s.m2[yb * s.W + xb] : 0.f;
        const float v = s.m2[p];
        if (v > behind && v >= ahead) cls = v > s.high * s.high ? 2 : (v > s.low * s.low ? 1 : 0);
    }
    m |= cls == 2 ? kStrong : cls == 1 ? kWeak : 0;
    s.meta[p] = m;
    s.parent[p] = cls ? p : -1;
}

__global__ __launch_bounds__(kBlock) void k_uf_union_edges(SegDev s) {
    int x, y;
    if (!pix(s, x, y)) return;
    const int p = y * s.W + x;
    if (s.parent[p] < 0) return;
    const int dx[4] = {1, -1, 0, 1}, dy[4] = {0, 1, 1, 1};  // E, SW, S, SE
    for (int k = 0; k < 4; ++k) {
        const int xx = x + dx[k], yy = y + dy[k];
        if (xx < 0 || xx >= s.W || yy >= s.H) continue;
        const int q = yy * s.W + xx;
        if (s.meta[q] & (kWeak | kStrong)) uf_unite(s.parent, p, q);
    }
}

__global__ __launch_bounds__(kBlock) void k_seg_strong(SegDev s) {
    int x, y;
    if (!pix(s, x, y)) return;
    const int p = y * s.W + x;
    if (s.meta[p] & kStrong) s.strong[uf_find(s.parent, p)] = 1;
}

__global__ __launch_bounds__(kBlock) void k_seg_edge(SegDev s) {
    int x, y;
    if (!pix(s, x, y)) return;
    const int p = y * s.W + x;
    const uint8_t m = s.meta[p];
    const bool e = (m & (kWeak | kStrong)) && s.strong[uf_find(s.parent, p)];
    if (e) s.meta[p] = m | kEdge;
    if (s.edges) s.edges[y * s.pitch + x] = e ? 1 : 0;
}

// Region pixels: valid normal, no barrier, no edge pixel in the 3x3 window.
__global__ __launch_bounds__(kBlock) void k_seg_rinit(SegDev s) {
    int x, y;
    if (!pix(s, x, y)) return;
    const int p = y * s.W + x;
    bool in = (s.valid[y * s.pitch + x] & 2) && !(s.meta[p] & kBarrier);
    for (int dv = -1; dv <= 1 && in; ++dv)
        for (int du = -1; du <= 1; ++du) {
            const int xx = x + du, yy = y + dv;
            if (xx >= 0 && xx < s.W && yy >= 0 && yy < s.H && (s.meta[yy * s.W + xx] & kEdge)) in = false;
        }
    s.parent2[p] = in ? p : -1;
    s.cnt[p] = 0;
    s.rank[p] = -1;
}

__global__ __launch_bounds__(kBlock) void k_uf_union_regions(SegDev s) {
    int x, y;
    if (!pix(s, x, y)) return;
    const int p = y * s.W + x;
    if (s.parent2[p] < 0) return;
    if (x + 1 < s.W && s.parent2[p + 1] >= 0) uf_unite(s.parent2, p, p + 1);
    if (y + 1 < s.H && s.parent2[p + s.W] >= 0) uf_unite(s.parent2, p, p + s.W);
}

// Component sizes: one atomic add per distinct root in each wave (the pixels
// of a wave mostly share one).
__global__ __launch_bounds__(kBlock) void k_seg_count(SegDev s) {
    int x = 0, y = 0;
    const bool in = pix(s, x, y);
    const int p = y * s.W + x;
    int r = -1;
    if (in && s.parent2[p] >= 0) r = uf_find(s.parent2, p);
    if (in) s.root[p] = r;
    unsigned long long pending = __ballot(r >= 0);
    while (pending) {  // wave-uniform: one pass per distinct root
        const int leader = __ffsll(pending) - 1;
        const int R = __shfl(r, leader);
        const unsigned long long m = __ballot(r == R);
        if ((int)(threadIdx.x & 63) == leader) atomicAdd(&s.cnt[R], __popcll(m));
        pending &= ~m;
    }
}

__global__ __launch_bounds__(kBlock) void k_seg_cand(SegDev s) {
    int x, y;
    if (!pix(s, x, y)) return;
    const int p = y * s.W + x;
    if (s.root[p] != p || s.cnt[p] < s.min_area) return;
    const int i = atomicAdd(s.ncand, 1);
    // larger key = larger component, then smaller root index
    s.cand[i] = ((unsigned long long)(uint32_t)s.cnt[p] << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)p);
}

// One block: bitonic sort of the candidates (descending) in LDS, then ranks.
__global__ __launch_bounds__(kBlock) void k_seg_sort(SegDev s) {
    __shared__ unsigned long long key[kSegMaxCand];
    const int n = *s.ncand;
    int m = 1;
    while (m < n) m <<= 1;
    for (int i = threadIdx.x; i < m; i += kBlock) key[i] = i < n ? s.cand[i] : 0ull;
    __syncthreads();
    for (int k = 2; k <= m; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < m; i += kBlock) {
                const int l = i ^ j;
                if (l > i) {
                    const bool desc = (i & k) == 0;
                    const unsigned long long a = key[i], b = key[l];
                    if (desc ? a < b : a > b) {
                        key[i] = b;
                        key[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    const int nr = min(n, s.max_regions);
    for (int i = threadIdx.x; i < nr; i += kBlock) {
        const int root = (int)(0xFFFFFFFFu - (uint32_t)(key[i] & 0xFFFFFFFFull));
        s.rank[root] = i;
    }
    if (threadIdx.x == 0) *s.n_regions = nr;
}

__global__ __launch_bounds__(kBlock) void k_seg_label(SegDev s) {
    int x, y;
    if (!pix(s, x, y)) return;
    const int p = y * s.W + x;
    const int r = s.root[p];
    s.region[y * s.pitch + x] = (int16_t)(r >= 0 ? s.rank[r] : -1);
}

template <typename T>
T* carve(uintptr_t& p, size_t n) {
    T* q = reinterpret_cast<T*>(p);
    p += (n * sizeof(T) + 255) & ~size_t(255);
    return q;
}

}  // namespace

size_t seg_bind_scratch(SegDev& s, void* scratch) {
    const uintptr_t base = reinterpret_cast<uintptr_t>(scratch);
    uintptr_t p = base;
    const size_t n = (size_t)s.W * s.H;
    s.m2 = carve<float>(p, n);
    s.root = reinterpret_cast<int32_t*>(s.m2);  // m2 is dead once suppression is done
    s.meta = carve<uint8_t>(p, n);
    s.strong = carve<uint8_t>(p, n);
    s.parent = carve<int32_t>(p, n);
    s.parent2 = carve<int32_t>(p, n);
    s.cnt = carve<int32_t>(p, n);
    s.rank = carve<int32_t>(p, n);
    s.cand = carve<unsigned long long>(p, kSegMaxCand);
    s.ncand = carve<int32_t>(p, 1);
    return (size_t)(p - base);
}

size_t seg_scratch_bytes(int W, int H) {
    SegDev s{};
    s.W = W;
    s.H = H;
    return seg_bind_scratch(s, nullptr);
}

hipError_t launch_segment(const SegDev& s, hipStream_t st) {
    const dim3 grid((s.W * s.H + kBlock - 1) / kBlock), blk(kBlock);
    hipLaunchKernelGGL(k_seg_grad, grid, blk, 0, st, s);
    hipLaunchKernelGGL(k_seg_nms, grid, blk, 0, st, s);
    hipLaunchKernelGGL(k_uf_union_edges, grid, blk, 0, st, s);
    hipLaunchKernelGGL(k_seg_strong, grid, blk, 0, st, s);
    hipLaunchKernelGGL(k_seg_edge, grid, blk, 0, st, s);
    hipLaunchKernelGGL(k_seg_rinit, grid, blk, 0, st, s);
    hipLaunchKernelGGL(k_uf_union_regions, grid, blk, 0, st, s);
    hipLaunchKernelGGL(k_seg_count, grid, blk, 0, st, s);
    hipLaunchKernelGGL(k_seg_cand, grid, blk, 0, st, s);
    hipLaunchKernelGGL(k_seg_sort, dim3(1), blk, 0, st, s);
    hipLaunchKernelGGL(k_seg_label, grid, blk, 0, st, s);
    return hipGetLastError();
}

}  // namespace ppk
