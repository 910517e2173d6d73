// Region contours simplified into polygons (Sec. III-D: the contours of the
// segmented normal image are simplified into polygons).  Host code over a
// host copy of the region label image:
//   - the contour of region g is its outer boundary: Moore-neighbourhood
//     tracing, clockwise on screen (y down), from the region's first pixel in
//     row-major order entered from the west, until the trace is back on the
//     start pixel and its next move would repeat the first move;
//   - Douglas-Peucker simplification of the closed contour, split at the
//     contour point farthest from the start (the first such); a point stays
//     iff its distance to the current chord exceeds eps pixels.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "pp.h"

namespace {

struct Px {
    int x, y;
};

// W, NW, N, NE, E, SE, S, SW
constexpr int kDx[8] = {-1, -1, 0, 1, 1, 1, 0, -1};
constexpr int kDy[8] = {0, -1, -1, -1, 0, 1, 1, 1};

struct Labels {
    const int16_t* p;
    int W, H, pitch;
    bool is(int x, int y, int g) const { return x >= 0 && x < W && y >= 0 && y < H && p[(size_t)y * pitch + x] == g; }
};

void trace(const Labels& L, int g, Px s, std::vector<Px>& out, size_t cap) {
    out.clear();
    out.push_back(s);
    Px c = s, first{-1, -1};
    int back = 0;  // direction from c to the last outside pixel checked: the start is entered from the west
    for (size_t step = 0; step < cap; ++step) {
        int dir = -1;
        for (int k = 1; k <= 8 && dir < 0; ++k) {
            const int d = (back + k) & 7;
            if (L.is(c.x + kDx[d], c.y + kDy[d], g)) dir = d;
        }
        if (dir < 0) return;  // a single pixel
        const int od = (dir + 7) & 7;
        const Px outside{c.x + kDx[od], c.y + kDy[od]};
        const Px next{c.x + kDx[dir], c.y + kDy[dir]};
        if (step == 0) {
            first = next;
        } else if (c.x == s.x && c.y == s.y && next.x == first.x && next.y == first.y) {
            out.pop_back();  // back on the start, about to repeat the first move: the contour is closed
            return;
        }
        int nb = 0;
        for (int d = 0; d < 8; ++d)
            if (next.x + kDx[d] == outside.x && next.y + kDy[d] == outside.y) nb = d;
        out.push_back(next);
        c = next;
        back = nb;
    }
}

// Douglas-Peucker over chain[0..n-1]; appends the kept points except the last to out.
void simplify(const std::vector<Px>& chain, double eps, std::vector<Px>& out) {
    const int n = (int)chain.size();
    std::vector<uint8_t> keep(n, 0);
    keep[0] = keep[n - 1] = 1;
    std::vector<std::pair<int, int>> todo{{0, n - 1}};
    while (!todo.empty()) {
        const auto [lo, hi] = todo.back();
        todo.pop_back();
        if (hi - lo < 2) continue;
        // distance of each point to the chord lo-hi, |cross| / len (to the point lo if the
        // chord is empty); the first farthest point splits.  The cross products (and the
        // squared distances) are exact integers, and distinct ones keep their order after
        // the division by len (the square root), so the search runs on the integers and
        // only the farthest point's distance is formed.
        const Px a = chain[lo], b = chain[hi];
        const int64_t ix = b.x - a.x, iy = b.y - a.y;
        const bool empty = ix == 0 && iy == 0;
        int64_t bestk = -1;
        int at = -1;
        for (int i = lo + 1; i < hi; ++i) {
            const Px& p = chain[i];
            const int64_t px = p.x - a.x, py = p.y - a.y;
            int64_t k = empty ? px * px + py * py : ix * py - iy * px;
            if (k < 0) k = -k;
            if (k > bestk) {
                bestk = k;
                at = i;
            }
        }
        const double dx = (double)ix, dy = (double)iy;
        const double best = empty ? std::sqrt((double)bestk) : (double)bestk / std::sqrt(dx * dx + dy * dy);
        if (best > eps) {
            keep[at] = 1;
            todo.push_back({lo, at});
            todo.push_back({at, hi});
        }
    }
    for (int i = 0; i + 1 < n; ++i)
        if (keep[i]) out.push_back(chain[i]);
}

}  // namespace

extern "C" pp_status pp_region_polygons(const int16_t* region_host, pp_frame_desc desc, int32_t n_regions,
                                        double eps_px, int32_t* xy_host, int32_t max_vertices,
                                        int32_t* offsets_host) {
    if (!region_host || !offsets_host || n_regions < 0 || n_regions > 32767 || !(eps_px >= 0.0) ||
        max_vertices < 0 || (max_vertices > 0 && !xy_host) || desc.width < 1 || desc.height < 1 ||
        desc.pitch_px < desc.width)
        return PP_E_INVAL;
    const Labels L{region_host, desc.width, desc.height, desc.pitch_px};
    std::vector<Px> first(n_regions, Px{-1, -1});
    int left = n_regions;
    for (int y = 0; y < L.H && left > 0; ++y) {
        const int16_t* row = region_host + (size_t)y * L.pitch;
        for (int x = 0; x < L.W && left > 0;) {
            const int g = row[x];
            if (g >= 0 && g < n_regions && first[g].x < 0) {
                first[g] = {x, y};
                --left;
            }
            // the rest of this run carries the same label: four labels per 64-bit compare
            const uint64_t rep = (uint64_t)(uint16_t)g * 0x0001000100010001ull;
            int e = x + 1;
            for (uint64_t v; e + 4 <= L.W; e += 4) {
                std::memcpy(&v, row + e, 8);
                if (v != rep) break;
            }
            while (e < L.W && row[e] == g) ++e;
            x = e;
        }
    }
    const size_t cap = 4 * (size_t)L.W * L.H + 8;
    std::vector<Px> contour, poly, chain;
    int64_t total = 0;
    for (int g = 0; g < n_regions; ++g) {
        offsets_host[g] = (int32_t)total;
        if (first[g].x < 0) continue;
        trace(L, g, first[g], contour, cap);
        poly.clear();
        const int m = (int)contour.size();
        if (m <= 2) {
            poly = contour;
        } else {
            // the first contour point farthest from the start (squared distances are exact
            // integers, and distinct ones keep their order under the square root)
            const Px s = contour[0];
            int far = 0;
            int64_t fd = -1;
            for (int i = 1; i < m; ++i) {
                const int64_t ex = contour[i].x - s.x, ey = contour[i].y - s.y;
                const int64_t d = ex * ex + ey * ey;
                if (d > fd) {
                    fd = d;
                    far = i;
                }
            }
            chain.assign(contour.begin(), contour.begin() + far + 1);
            simplify(chain, eps_px, poly);
            chain.assign(contour.begin() + far, contour.end());
            chain.push_back(s);
            simplify(chain, eps_px, poly);
        }
        for (const Px& p : poly) {
            if (total < max_vertices) {
                xy_host[2 * total] = p.x;
                xy_host[2 * total + 1] = p.y;
            }
            ++total;
        }
    }
    offsets_host[n_regions] = total > INT32_MAX ? INT32_MAX : (int32_t)total;
    return total > max_vertices ? PP_E_NOMEM : PP_OK;
}
