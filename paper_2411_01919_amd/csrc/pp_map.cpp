// Polygon map with vertical drift compensation (Sec. III-E, Eqs. 4-10),
// host code in float64.
//
// Each frame brings polygons observed in the camera frame (plane, centroid,
// support, and the pixel polygon that pp_region_polygons extracted, lifted
// onto the plane through the intrinsics) and the camera pose from odometry,
// whose height drifts.  The map keeps near-horizontal polygons (normal within
// max_tilt of world +Z): heights and vertical drift concern steppable
// surfaces.  Per frame:
//   - raw heights: world z of each polygon's centroid under the given pose;
//   - matching (Eqs. 4-5): a polygon matches the map polygon whose footprint
//     (convex hull in world x, y) overlaps its own with positive area and
//     whose height is within the drift tolerance of the raw height minus the
//     current drift estimate; the smallest height difference wins (ties: the
//     older map polygon);
//   - measurement: the mean of raw height minus map height over the matches;
//     the scalar Kalman filter of the drift (Eqs. 6-10) then predicts and,
//     with a measurement, updates;
//   - the polygons, corrected by the updated estimate, are merged into their
//     match (footprint: hull of both; height: support-weighted mean) or
//     appended, in input order.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "pp.h"

namespace {

struct V2 {
    double x, y;
};

double cross(const V2& o, const V2& a, const V2& b) { return (a.x - o.x) * (b.y - o.y) - (a.y - o.y) * (b.x - o.x); }

// Counter-clockwise convex hull (Andrew's monotone chain), collinear points dropped.
std::vector<V2> hull_of(std::vector<V2> p) {
    std::sort(p.begin(), p.end(), [](const V2& a, const V2& b) { return a.x < b.x || (a.x == b.x && a.y < b.y); });
    p.erase(std::unique(p.begin(), p.end(), [](const V2& a, const V2& b) { return a.x == b.x && a.y == b.y; }),
            p.end());
    if (p.size() < 3) return p;
    std::vector<V2> h(2 * p.size());
    size_t k = 0;
    for (size_t i = 0; i < p.size(); ++i) {
        while (k >= 2 && cross(h[k - 2], h[k - 1], p[i]) <= 0) --k;
        h[k++] = p[i];
    }
    for (size_t i = p.size() - 1, t = k + 1; i-- > 0;) {
        while (k >= t && cross(h[k - 2], h[k - 1], p[i]) <= 0) --k;
        h[k++] = p[i];
    }
    h.resize(k - 1);
    return h;
}

// Separating-axis test: do two counter-clockwise convex polygons overlap with
// positive area?  Projections that only touch count as separated.
bool overlaps(const std::vector<V2>& a, const std::vector<V2>& b) {
    if (a.size() < 3 || b.size() < 3) return false;
    const std::vector<V2>* polys[2] = {&a, &b};
    for (const auto* P : polys) {
        const size_t n = P->size();
        for (size_t i = 0; i < n; ++i) {
            const V2 &p = (*P)[i], &q = (*P)[(i + 1) % n];
            const double ax = -(q.y - p.y), ay = q.x - p.x;  // edge normal
            double amin = INFINITY, amax = -INFINITY, bmin = INFINITY, bmax = -INFINITY;
            for (const V2& v : a) {
                const double s = ax * v.x + ay * v.y;
                amin = std::min(amin, s);
                amax = std::max(amax, s);
            }
            for (const V2& v : b) {
                const double s = ax * v.x + ay * v.y;
                bmin = std::min(bmin, s);
                bmax = std::max(bmax, s);
            }
            if (amax <= bmin || bmax <= amin) return false;
        }
    }
    return true;
}

struct MapPoly {
    double height;
    int64_t support;
    std::vector<V2> hull;
};

struct Cand {
    bool horizontal;
    double z_raw;
    int64_t support;
    std::vector<V2> hull;
};

}  // namespace

struct pp_map {
    pp_map_params prm;
    double cos_tilt;
    double x = 0.0;  // drift estimate
    double P = 0.0;  // its variance
    std::vector<MapPoly> polys;
};

extern "C" {

pp_status pp_map_create(const pp_map_params* p, pp_map** out) {
    if (!p || !out || !(p->drift_tolerance_m > 0.0) || !(p->sigma_p >= 0.0) || !(p->sigma_m > 0.0) ||
        !(p->max_tilt_deg >= 0.0 && p->max_tilt_deg < 90.0) || !std::isfinite(p->sigma_p))
        return PP_E_INVAL;
    pp_map* m = new (std::nothrow) pp_map;
    if (!m) return PP_E_NOMEM;
    m->prm = *p;
    m->cos_tilt = std::cos(p->max_tilt_deg * M_PI / 180.0);
    *out = m;
    return PP_OK;
}

pp_status pp_map_destroy(pp_map* m) {
    delete m;
    return PP_OK;
}

pp_status pp_map_integrate(pp_map* m, pp_intrinsics K, const double* R, const double* C, const pp_map_observation* obs,
                           int32_t n, int32_t* match_of, pp_map_frame_result* out) {
    if (!m || !R || !C || !out || n < 0 || (n > 0 && !obs) || !(K.fx > 0.f) || !(K.fy > 0.f)) return PP_E_INVAL;
    for (int32_t i = 0; i < n; ++i)
        if (obs[i].n_vertices < 0 || (obs[i].n_vertices > 0 && !obs[i].xy_px) || obs[i].support < 0) return PP_E_INVAL;
    auto rot = [&](const double v[3], double w[3]) {
        for (int r = 0; r < 3; ++r) w[r] = R[3 * r] * v[0] + R[3 * r + 1] * v[1] + R[3 * r + 2] * v[2];
    };
    std::vector<Cand> cands(n);
    for (int32_t i = 0; i < n; ++i) {
        const pp_map_observation& o = obs[i];
        double nw[3];
        rot(o.n, nw);
        Cand& c = cands[i];
        c.horizontal = std::fabs(nw[2]) >= m->cos_tilt;
        if (!c.horizontal) continue;
        double cw[3];
        rot(o.centroid, cw);
        c.z_raw = cw[2] + C[2];
        c.support = o.support;
        std::vector<V2> pts;
        for (int32_t v = 0; v < o.n_vertices; ++v) {
            // the pixel's ray (x = column, y = row) meets the plane n.p + d = 0
            const double ray[3] = {(o.xy_px[2 * v] - (double)K.cx) / K.fx, (o.xy_px[2 * v + 1] - (double)K.cy) / K.fy,
                                   1.0};
            const double nr = o.n[0] * ray[0] + o.n[1] * ray[1] + o.n[2] * ray[2];
            if (nr == 0.0) continue;
            const double t = -o.d / nr;
            const double pc[3] = {t * ray[0], t * ray[1], t * ray[2]};
            double pw[3];
            rot(pc, pw);
            pts.push_back({pw[0] + C[0], pw[1] + C[1]});
        }
        c.hull = hull_of(std::move(pts));
    }
    // matching against the map as it stands, heights corrected by the current estimate
    std::vector<int32_t> match(n, -2);
    double msum = 0.0;
    int matched = 0, skipped = 0;
    for (int32_t i = 0; i < n; ++i) {
        const Cand& c = cands[i];
        if (!c.horizontal) {
            ++skipped;
            continue;
        }
        const double zc = c.z_raw - m->x;
        double best = INFINITY;
        int bj = -1;
        for (size_t j = 0; j < m->polys.size(); ++j) {
            const double dz = std::fabs(zc - m->polys[j].height);
            if (dz <= m->prm.drift_tolerance_m && dz < best && overlaps(c.hull, m->polys[j].hull)) {
                best = dz;
                bj = (int)j;
            }
        }
        match[i] = bj;
        if (bj >= 0) {
            msum += c.z_raw - m->polys[bj].height;
            ++matched;
        }
    }
    // Eqs. 6-10: x_{k|k-1} = x_{k-1}, P_{k|k-1} = P_{k-1} + sigma_p; with a measurement
    // K = P_{k|k-1} / (P_{k|k-1} + sigma_m), x_k = x_{k|k-1} + K (z_k - x_{k|k-1}), P_k = (1 - K) P_{k|k-1}
    const double P_pred = m->P + m->prm.sigma_p;
    double meas = NAN;
    if (matched > 0) {
        meas = msum / matched;
        const double gain = P_pred / (P_pred + m->prm.sigma_m);
        m->x = m->x + gain * (meas - m->x);
        m->P = (1.0 - gain) * P_pred;
    } else {
        m->P = P_pred;
    }
    int added = 0;
    for (int32_t i = 0; i < n; ++i) {
        Cand& c = cands[i];
        if (!c.horizontal) continue;
        const double z = c.z_raw - m->x;
        if (match[i] >= 0) {
            MapPoly& mp = m->polys[match[i]];
            mp.height = (mp.height * (double)mp.support + z * (double)c.support) / (double)(mp.support + c.support);
            mp.support += c.support;
            std::vector<V2> both = mp.hull;
            both.insert(both.end(), c.hull.begin(), c.hull.end());
            mp.hull = hull_of(std::move(both));
        } else {
            m->polys.push_back(MapPoly{z, c.support, std::move(c.hull)});
            ++added;
        }
    }
    if (match_of)
        for (int32_t i = 0; i < n; ++i) match_of[i] = match[i];
    out->matched = matched;
    out->added = added;
    out->skipped = skipped;
    out->pad = 0;
    out->measurement = meas;
    out->drift = m->x;
    out->variance = m->P;
    return PP_OK;
}

pp_status pp_map_size(const pp_map* m, int32_t* n) {
    if (!m || !n) return PP_E_INVAL;
    *n = (int32_t)m->polys.size();
    return PP_OK;
}

pp_status pp_map_polygon(const pp_map* m, int32_t i, pp_map_polygon_info* info, double* xy, int32_t max_vertices) {
    if (!m || !info || i < 0 || i >= (int32_t)m->polys.size() || max_vertices < 0 || (max_vertices > 0 && !xy))
        return PP_E_INVAL;
    const MapPoly& p = m->polys[i];
    info->height = p.height;
    info->support = p.support;
    info->n_vertices = (int32_t)p.hull.size();
    info->pad = 0;
    for (int32_t v = 0; v < info->n_vertices && v < max_vertices; ++v) {
        xy[2 * v] = p.hull[v].x;
        xy[2 * v + 1] = p.hull[v].y;
    }
    return info->n_vertices > max_vertices ? PP_E_NOMEM : PP_OK;
}

}  // extern "C"
