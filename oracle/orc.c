/*
 * CPU FP64 oracle of the plane-extraction path of arXiv 2411.01919.
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow reference that the GPU library is
 * checked against.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code with the GPU library.
 *
 * Written for reading against the paper, not for speed: every step is the
 * plain definition, in float64, in the order the method states it.  OpenMP
 * is used only across independent pixels or hypotheses; every reduction is
 * either an integer count or done serially in a fixed order.
 *
 * Readings of the paper taken here (the paper is silent or garbled on them):
 *  - holes: depth 0 is "no measurement"; they get no flux and stay 0;
 *  - diffusion: the per-edge flux form of Eq. 1 on the 4-neighbourhood (the
 *    classical explicit Perona-Malik scheme), gradient along an edge taken as
 *    the neighbour difference, zero flux across the border and into holes,
 *    Jacobi update (every pixel reads the previous iterate);
 *  - normals: Eq. 2 taken as the geometric normal of the back-projected
 *    surface: Sobel sums of the point image, n = -(Gx x Gy)/|Gx x Gy|, which
 *    faces the camera;
 *  - RANSAC: whole-frame sequential extraction; the hypothesis with the most
 *    inliers wins (ties to the lowest index); one total-least-squares refit on
 *    its inliers; the refit plane's inliers are removed and labelled if there
 *    are at least min_inliers of them; strict "<" against the threshold;
 *  - sampling: Philox4x64-10 keyed by (seed, frame) with counter
 *    (hypothesis, round, block, 0); each 64-bit word w picks position
 *    floor(w * M0 / 2^64) in the frame's fixed list of valid pixels and is
 *    rejected if that pixel is already assigned or already chosen; 16 blocks
 *    (64 words) at most, else the hypothesis is invalid; a triple whose
 *    cross product is at most 1e-3 |e1| |e2| is degenerate (invalid).
 */
#include "orc.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11): 10 rounds of the 4x64 S-box with the
 * published multipliers and Weyl key increments.                           */
/* ------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t MUL0 = 0xD2E7470EE14C6C93ULL, MUL1 = 0xCA5A826395121157ULL;
    const uint64_t WEYL0 = 0x9E3779B97F4A7C15ULL, WEYL1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += WEYL0;
            k1 += WEYL1;
        }
        unsigned __int128 p0 = (unsigned __int128)MUL0 * c0;
        unsigned __int128 p1 = (unsigned __int128)MUL1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Eq. 1 / Alg. 1: explicit Perona-Malik diffusion.                          */
/* I^{it+1}_p = I^it_p + lambda * sum_{q in N4(p), inside, valid} g(I_q - I_p) (I_q - I_p) */
/* ------------------------------------------------------------------------ */
static double edge_stop_g(double x, double kappa, int kind) {
    double s = x / kappa;
    if (kind == 1) return 1.0 / (1.0 + s * s);
    return exp(-(s * s));
}

void orc_diffuse(const double* depth, int W, int H, int iters, double lambda, double kappa,
                 int edge_stop, double* out) {
    size_t n = (size_t)W * H;
    double* cur = (double*)malloc(n * sizeof(double));
    double* nxt = (double*)malloc(n * sizeof(double));
    for (size_t p = 0; p < n; ++p) cur[p] = depth[p];
    const int du[4] = {0, 0, -1, 1};
    const int dv[4] = {-1, 1, 0, 0};
    for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(static)
        for (int v = 0; v < H; ++v) {
            for (int u = 0; u < W; ++u) {
                size_t p = (size_t)v * W + u;
                if (!(depth[p] > 0.0)) {
                    nxt[p] = 0.0;
                    continue;
                }
                double flux = 0.0;
                for (int k = 0; k < 4; ++k) {
                    int uq = u + du[k], vq = v + dv[k];
                    if (uq < 0 || uq >= W || vq < 0 || vq >= H) continue; /* zero flux at the border */
                    size_t q = (size_t)vq * W + uq;
                    if (!(depth[q] > 0.0)) continue;                       /* zero flux into a hole */
                    double delta = cur[q] - cur[p];
                    flux += edge_stop_g(delta, kappa, edge_stop) * delta;
                }
                nxt[p] = cur[p] + lambda * flux;
            }
        }
        double* t = cur; cur = nxt; nxt = t;
    }
    memcpy(out, cur, n * sizeof(double));
    free(cur);
    free(nxt);
}

/* ------------------------------------------------------------------------ */
/* Diffusion variants beside the hot path's conservative 4-neighbour form.   */
/*  scheme 1: Alg. 1 as printed, pixel-centred: c_p = g(|grad I_p|) with the */
/*            gradient from central differences (one-sided next to a hole or */
/*            the border, 0 with no neighbour on either side), then          */
/*            I_p += lambda c_p lap(I)_p, lap = sum over valid 4-neighbours    */
/*            of (I_q - I_p).  Not conservative.                              */
/*  scheme 2: per-edge flux over the 8-neighbourhood: diagonal neighbours at  */
/*            distance sqrt(2) with weight 1/2: I_p += lambda sum_q w_q       */
/*            g(|I_q - I_p| / d_q) (I_q - I_p).  Conservative; stable for     */
/*            lambda <= 1/6.                                                 */
/* ------------------------------------------------------------------------ */
void orc_diffuse_variant(const double* depth, int W, int H, int iters, double lambda, double kappa,
                         int edge_stop, int scheme, double* out) {
    size_t n = (size_t)W * H;
    double* cur = (double*)malloc(n * sizeof(double));
    double* nxt = (double*)malloc(n * sizeof(double));
    for (size_t p = 0; p < n; ++p) cur[p] = depth[p];
#define VALID(u, v) ((u) >= 0 && (u) < W && (v) >= 0 && (v) < H && depth[(size_t)(v) * W + (u)] > 0.0)
#define VAL(u, v) cur[(size_t)(v) * W + (u)]
    for (int it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(static)
        for (int v = 0; v < H; ++v) {
            for (int u = 0; u < W; ++u) {
                size_t p = (size_t)v * W + u;
                if (!(depth[p] > 0.0)) {
                    nxt[p] = 0.0;
                    continue;
                }
                double Ip = cur[p];
                if (scheme == 1) {
                    int e = VALID(u + 1, v), w = VALID(u - 1, v), s = VALID(u, v + 1), nn = VALID(u, v - 1);
                    double gx = e && w ? (VAL(u + 1, v) - VAL(u - 1, v)) / 2.0 : e ? VAL(u + 1, v) - Ip : w ? Ip - VAL(u - 1, v) : 0.0;
                    double gy = s && nn ? (VAL(u, v + 1) - VAL(u, v - 1)) / 2.0 : s ? VAL(u, v + 1) - Ip : nn ? Ip - VAL(u, v - 1) : 0.0;
                    double lap = 0.0;
                    if (e) lap += VAL(u + 1, v) - Ip;
                    if (w) lap += VAL(u - 1, v) - Ip;
                    if (s) lap += VAL(u, v + 1) - Ip;
                    if (nn) lap += VAL(u, v - 1) - Ip;
                    double c = edge_stop_g(sqrt(gx * gx + gy * gy), kappa, edge_stop);
                    nxt[p] = Ip + lambda * c * lap;
                } else {
                    double flux = 0.0;
                    for (int dv = -1; dv <= 1; ++dv)
                        for (int du = -1; du <= 1; ++du) {
                            if (!du && !dv) continue;
                            if (!VALID(u + du, v + dv)) continue;
                            int diag = du && dv;
                            double delta = VAL(u + du, v + dv) - Ip;
                            double dist = diag ? sqrt(2.0) : 1.0;
                            double wq = diag ? 0.5 : 1.0;
                            flux += wq * edge_stop_g(fabs(delta) / dist, kappa, edge_stop) * delta;
                        }
                    nxt[p] = Ip + lambda * flux;
                }
            }
        }
        double* t = cur; cur = nxt; nxt = t;
    }
#undef VALID
#undef VAL
    memcpy(out, cur, n * sizeof(double));
    free(cur);
    free(nxt);
}

/* ------------------------------------------------------------------------ */
/* Back-projection (Sec. III-D: polygons projected to 3-D with K; Alg. 2).    */
/* ------------------------------------------------------------------------ */
void orc_backproject(const double* depth_mm, int W, int H, double fx, double fy, double cx, double cy,
                     double* P, uint8_t* valid) {
    size_t n = (size_t)W * H;
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            double z = depth_mm[p] / 1000.0;
            int ok = depth_mm[p] > 0.0;
            valid[p] = (uint8_t)ok;
            P[p] = ok ? z * ((double)u - cx) / fx : 0.0;
            P[n + p] = ok ? z * ((double)v - cy) / fy : 0.0;
            P[2 * n + p] = ok ? z : 0.0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Eq. 2 / Alg. 1: Sobel gradients and the normal image.                      */
/* ------------------------------------------------------------------------ */
void orc_normals(const double* P, const uint8_t* valid, int W, int H, double* N, uint8_t* nvalid,
                 double* gx_out, double* gy_out) {
    const double SX[3][3] = {{-1, 0, 1}, {-2, 0, 2}, {-1, 0, 1}};
    const double SY[3][3] = {{-1, -2, -1}, {0, 0, 0}, {1, 2, 1}};
    size_t n = (size_t)W * H;
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v) {
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            int ok = (u >= 1 && u <= W - 2 && v >= 1 && v <= H - 2);
            for (int j = 0; ok && j < 3; ++j)
                for (int i = 0; ok && i < 3; ++i)
                    if (!valid[(size_t)(v + j - 1) * W + (u + i - 1)]) ok = 0;
            double gx[3] = {0, 0, 0}, gy[3] = {0, 0, 0};
            if (ok) {
                for (int j = 0; j < 3; ++j)
                    for (int i = 0; i < 3; ++i) {
                        size_t q = (size_t)(v + j - 1) * W + (u + i - 1);
                        for (int c = 0; c < 3; ++c) {
                            gx[c] += SX[j][i] * P[c * n + q];
                            gy[c] += SY[j][i] * P[c * n + q];
                        }
                    }
            }
            double m[3] = {gx[1] * gy[2] - gx[2] * gy[1], gx[2] * gy[0] - gx[0] * gy[2],
                           gx[0] * gy[1] - gx[1] * gy[0]};
            double mn = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
            if (!(mn > 0.0)) ok = 0;
            nvalid[p] = (uint8_t)ok;
            for (int c = 0; c < 3; ++c) {
                N[c * n + p] = ok ? -m[c] / mn : 0.0;
                if (gx_out) gx_out[c * n + p] = gx[c];
                if (gy_out) gy_out[c * n + p] = gy[c];
            }
        }
    }
}

int orc_valid_list(const uint8_t* valid, int npx, int32_t* L) {
    int m = 0;
    for (int p = 0; p < npx; ++p)
        if (valid[p]) L[m++] = p;
    return m;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2: the random choice of 3 points and the plane through them.       */
/* ------------------------------------------------------------------------ */
static void point_at(const double* P, size_t n, int px, double out[3]) {
    out[0] = P[px];
    out[1] = P[n + px];
    out[2] = P[2 * n + px];
}

void orc_hypotheses(const double* P, int W, int H, const int32_t* L, int M0, const uint8_t* assigned,
                    const orc_ransac_params* prm, int r, int32_t* triples, double* planes, uint8_t* hvalid) {
    size_t n = (size_t)W * H;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < prm->hyps; ++j) {
        int slot[3] = {-1, -1, -1};
        int got = 0;
        for (int b = 0; b < 16 && got < 3; ++b) {
            uint64_t ctr[4] = {(uint64_t)j, (uint64_t)r, (uint64_t)b, 0};
            uint64_t key[2] = {prm->seed, prm->frame};
            uint64_t w[4];
            orc_philox4x64_10(ctr, key, w);
            for (int q = 0; q < 4 && got < 3; ++q) {
                int k = (int)(((unsigned __int128)w[q] * (uint64_t)M0) >> 64);
                if (assigned[L[k]]) continue;
                int dup = 0;
                for (int s = 0; s < got; ++s)
                    if (slot[s] == k) dup = 1;
                if (dup) continue;
                slot[got++] = k;
            }
        }
        double* pl = planes + 4 * (size_t)j;
        pl[0] = pl[1] = pl[2] = pl[3] = 0.0;
        triples[3 * j + 0] = slot[0];
        triples[3 * j + 1] = slot[1];
        triples[3 * j + 2] = slot[2];
        hvalid[j] = 0;
        if (got < 3) continue;
        double p0[3], p1[3], p2[3];
        point_at(P, n, L[slot[0]], p0);
        point_at(P, n, L[slot[1]], p1);
        point_at(P, n, L[slot[2]], p2);
        double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        double m[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
        double mn = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        double l2 = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
        if (!(mn > 1e-3 * l1 * l2)) continue; /* degenerate triple */
        double nn[3] = {m[0] / mn, m[1] / mn, m[2] / mn};
        double d = -(nn[0] * p0[0] + nn[1] * p0[1] + nn[2] * p0[2]);
        if (d < 0) {
            nn[0] = -nn[0]; nn[1] = -nn[1]; nn[2] = -nn[2];
            d = -d;
        }
        pl[0] = nn[0]; pl[1] = nn[1]; pl[2] = nn[2]; pl[3] = d;
        hvalid[j] = 1;
    }
}

/* Gather the unassigned valid points (positions of L in order). */
static int gather_remaining(const double* P, int W, int H, const int32_t* L, int M0, const uint8_t* assigned,
                            double* xyz, int32_t* pix) {
    size_t n = (size_t)W * H;
    int m = 0;
    for (int k = 0; k < M0; ++k) {
        int px = L[k];
        if (assigned[px]) continue;
        xyz[3 * (size_t)m + 0] = P[px];
        xyz[3 * (size_t)m + 1] = P[n + px];
        xyz[3 * (size_t)m + 2] = P[2 * n + px];
        pix[m] = px;
        ++m;
    }
    return m;
}

/* Alg. 2 inner loop: for every point, distance to the plane (Eq. 3), inlier iff below t. */
static void score_points(const double* xyz, int m, const double* planes, const uint8_t* hvalid, int nh,
                         double thresh, const double* eps, int32_t* counts, int32_t* counts_lo,
                         int32_t* counts_hi) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < nh; ++j) {
        int32_t c = 0, clo = 0, chi = 0;
        if (hvalid[j]) {
            const double* pl = planes + 4 * (size_t)j;
            double tlo = eps ? thresh - eps[j] : thresh;
            double thi = eps ? thresh + eps[j] : thresh;
            for (int i = 0; i < m; ++i) {
                const double* p = xyz + 3 * (size_t)i;
                double dist = fabs(pl[0] * p[0] + pl[1] * p[1] + pl[2] * p[2] + pl[3]);
                c += dist < thresh;
                clo += dist < tlo;
                chi += dist < thi;
            }
        }
        counts[j] = c;
        if (counts_lo) counts_lo[j] = clo;
        if (counts_hi) counts_hi[j] = chi;
    }
}

void orc_score(const double* P, int W, int H, const int32_t* L, int M0, const uint8_t* assigned,
               const double* planes, const uint8_t* hvalid, int nh, double thresh, const double* eps,
               int32_t* counts, int32_t* counts_lo, int32_t* counts_hi, double* pmax) {
    double* xyz = (double*)malloc(3 * (size_t)(M0 > 0 ? M0 : 1) * sizeof(double));
    int32_t* pix = (int32_t*)malloc((size_t)(M0 > 0 ? M0 : 1) * sizeof(int32_t));
    int m = gather_remaining(P, W, H, L, M0, assigned, xyz, pix);
    if (pmax) {
        double best = 0.0;
        for (int i = 0; i < m; ++i) {
            const double* p = xyz + 3 * (size_t)i;
            double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
            if (r > best) best = r;
        }
        *pmax = best;
    }
    score_points(xyz, m, planes, hvalid, nh, thresh, eps, counts, counts_lo, counts_hi);
    free(xyz);
    free(pix);
}

/* ------------------------------------------------------------------------ */
/* Symmetric 3x3 eigen-decomposition, cyclic Jacobi (Golub & Van Loan 8.5).  */
/* ------------------------------------------------------------------------ */
void orc_eig3(const double A_in[9], double w[3], double V[9]) {
    double A[3][3], Q[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            A[i][j] = A_in[3 * i + j];
            Q[i][j] = (i == j) ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off == 0.0 || off <= 1e-40 * dia) break;
        for (int p = 0; p < 2; ++p) {
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                /* rotation that zeroes A[p][q]: tan of the angle is the smaller root */
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0);
                double s = t * c;
                /* A <- J^T A J with J the (p,q) rotation [c s; -s c] */
                for (int k = 0; k < 3; ++k) {
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    double qkp = Q[k][p], qkq = Q[k][q];
                    Q[k][p] = c * qkp - s * qkq;
                    Q[k][q] = s * qkp + c * qkq;
                }
            }
        }
    }
    /* sort ascending */
    int idx[3] = {0, 1, 2};
    double ev[3] = {A[0][0], A[1][1], A[2][2]};
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (ev[idx[b]] < ev[idx[a]]) {
                int t = idx[a]; idx[a] = idx[b]; idx[b] = t;
            }
    for (int c = 0; c < 3; ++c) {
        w[c] = ev[idx[c]];
        for (int k = 0; k < 3; ++k) V[3 * k + c] = Q[k][idx[c]];
    }
}

/* Least-squares refit: the plane through the centroid whose normal is the
 * direction of least scatter minimises the sum of squared distances (the
 * best plane of Sec. III-A, Eq. 3 with a squared distance). */
int orc_refit(const double* P, int W, int H, const int32_t* idx, int cnt, double plane[4], double centroid[3]) {
    size_t n = (size_t)W * H;
    plane[0] = plane[1] = plane[2] = plane[3] = 0.0;
    centroid[0] = centroid[1] = centroid[2] = 0.0;
    if (cnt < 3) return -1;
    double c[3] = {0, 0, 0};
    for (int i = 0; i < cnt; ++i)
        for (int k = 0; k < 3; ++k) c[k] += P[k * n + idx[i]];
    for (int k = 0; k < 3; ++k) c[k] /= cnt;
    double C[9] = {0};
    for (int i = 0; i < cnt; ++i) {
        double q[3];
        for (int k = 0; k < 3; ++k) q[k] = P[k * n + idx[i]] - c[k];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) C[3 * a + b] += q[a] * q[b];
    }
    double w[3], V[9];
    orc_eig3(C, w, V);
    double nn[3] = {V[0], V[3], V[6]}; /* column 0: smallest eigenvalue */
    double nrm = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    for (int k = 0; k < 3; ++k) nn[k] /= nrm;
    double d = -(nn[0] * c[0] + nn[1] * c[1] + nn[2] * c[2]);
    if (d < 0) {
        for (int k = 0; k < 3; ++k) nn[k] = -nn[k];
        d = -d;
    }
    plane[0] = nn[0]; plane[1] = nn[1]; plane[2] = nn[2]; plane[3] = d;
    centroid[0] = c[0]; centroid[1] = c[1]; centroid[2] = c[2];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One round of sequential RANSAC (follow mode).                              */
/* ------------------------------------------------------------------------ */
void orc_ransac_round(const double* P, int W, int H, const int32_t* L, int M0, const uint8_t* assigned,
                      const orc_ransac_params* prm, int r, const double* eps,
                      int32_t* triples, double* planes, uint8_t* hvalid,
                      int32_t* counts, int32_t* counts_lo, int32_t* counts_hi,
                      uint8_t* smask, uint8_t* fmask, orc_round_result* res) {
    size_t n = (size_t)W * H;
    int nh = prm->hyps;
    memset(res, 0, sizeof(*res));
    res->jstar = -1;
    if (smask) memset(smask, 0, n);
    if (fmask) memset(fmask, 0, n);

    double* xyz = (double*)malloc(3 * (size_t)(M0 > 0 ? M0 : 1) * sizeof(double));
    int32_t* pix = (int32_t*)malloc((size_t)(M0 > 0 ? M0 : 1) * sizeof(int32_t));
    int m = gather_remaining(P, W, H, L, M0, assigned, xyz, pix);
    res->n_remaining = m;
    if (m < 3) {
        res->status = 3;
        free(xyz); free(pix);
        return;
    }

    int32_t* tr = triples ? triples : (int32_t*)malloc(3 * (size_t)nh * sizeof(int32_t));
    double* pl = planes ? planes : (double*)malloc(4 * (size_t)nh * sizeof(double));
    uint8_t* hv = hvalid ? hvalid : (uint8_t*)malloc((size_t)nh);
    int32_t* ct = counts ? counts : (int32_t*)malloc((size_t)nh * sizeof(int32_t));

    orc_hypotheses(P, W, H, L, M0, assigned, prm, r, tr, pl, hv);
    score_points(xyz, m, pl, hv, nh, prm->thresh, eps, ct, counts_lo, counts_hi);

    /* select: most inliers, ties to the lowest index, invalid never chosen */
    int js = -1;
    for (int j = 0; j < nh; ++j)
        if (hv[j] && (js < 0 || ct[j] > ct[js])) js = j;
    res->jstar = js;
    if (js < 0) {
        res->status = 1;
    } else {
        const double* h = pl + 4 * (size_t)js;
        memcpy(res->hyp_plane, h, 4 * sizeof(double));
        int32_t* S = (int32_t*)malloc((size_t)m * sizeof(int32_t));
        int ns = 0;
        for (int i = 0; i < m; ++i) {
            const double* p = xyz + 3 * (size_t)i;
            if (fabs(h[0] * p[0] + h[1] * p[1] + h[2] * p[2] + h[3]) < prm->thresh) {
                S[ns++] = pix[i];
                if (smask) smask[pix[i]] = 1;
            }
        }
        res->s_count = ns;
        orc_refit(P, W, H, S, ns, res->plane, res->centroid);
        const double* q = res->plane;
        int nf = 0;
        for (int i = 0; i < m; ++i) {
            const double* p = xyz + 3 * (size_t)i;
            if (fabs(q[0] * p[0] + q[1] * p[1] + q[2] * p[2] + q[3]) < prm->thresh) {
                ++nf;
                if (fmask) fmask[pix[i]] = 1;
            }
        }
        res->f_count = nf;
        res->status = (nf >= prm->min_inliers) ? 0 : 2;
        free(S);
    }
    if (!triples) free(tr);
    if (!planes) free(pl);
    if (!hvalid) free(hv);
    if (!counts) free(ct);
    free(xyz);
    free(pix);
}

int orc_ransac(const double* P, const uint8_t* valid, int W, int H, const orc_ransac_params* prm,
               int8_t* labels, double* planes_out, double* centroids_out, int32_t* inliers_out,
               int32_t* jstar_out, double* residuals) {
    size_t n = (size_t)W * H;
    int32_t* L = (int32_t*)malloc(n * sizeof(int32_t));
    int M0 = orc_valid_list(valid, (int)n, L);
    uint8_t* assigned = (uint8_t*)calloc(n, 1);
    uint8_t* fmask = (uint8_t*)malloc(n);
    for (size_t p = 0; p < n; ++p) labels[p] = -1;
    double res_count = 0.0;
    int np = 0;
    for (int r = 0; r < prm->max_planes; ++r) {
        orc_round_result rr;
        orc_ransac_round(P, W, H, L, M0, assigned, prm, r, NULL, NULL, NULL, NULL, NULL, NULL, NULL,
                         NULL, fmask, &rr);
        if (rr.status == 3) break;
        if (rr.status == 1) break;
        res_count += (double)rr.n_remaining * prm->hyps;
        if (rr.status != 0) break;
        for (size_t p = 0; p < n; ++p)
            if (fmask[p]) {
                labels[p] = (int8_t)np;
                assigned[p] = 1;
            }
        if (planes_out) memcpy(planes_out + 4 * (size_t)np, rr.plane, 4 * sizeof(double));
        if (centroids_out) memcpy(centroids_out + 3 * (size_t)np, rr.centroid, 3 * sizeof(double));
        if (inliers_out) inliers_out[np] = rr.f_count;
        if (jstar_out) jstar_out[np] = rr.jstar;
        ++np;
        if (rr.n_remaining - rr.f_count < 3) break;
    }
    if (residuals) *residuals = res_count;
    free(L);
    free(assigned);
    free(fmask);
    return np;
}

/* ------------------------------------------------------------------------ */
/* Region-mode RANSAC: Alg. 2 as printed, one region at a time.               */
/* For each region g (pixels with depth and region label g, 0 <= g < R, in    */
/* row-major order):                                                          */
/*  - hypothesis j draws three distinct positions of the region's list from  */
/*    Philox4x64-10 words, key (seed, frame), counter (j, g, b, 1), position */
/*    floor(w n_g / 2^64); a repeated position is skipped; a degenerate      */
/*    triple gives no plane;                                                 */
/*  - error_j = sum over all the region's points of |n.p + d| (Eq. 3),       */
/*    inliers_j = #{|n.p + d| < t};                                          */
/*  - the model kept is the first one with the smallest error (strict <, so  */
/*    ties go to the smaller j); none when no hypothesis has a plane;        */
/*  - it is stored iff inliers / n_g > 0.9, evaluated as 10 inliers > 9 n_g. */
/* labels[p] = g for the inliers of a stored model, -1 elsewhere;             */
/* centroids[g] = mean of those inliers.  Returns the number stored.         */
/* ------------------------------------------------------------------------ */
int orc_ransac_regions(const double* P, const uint8_t* valid, const int16_t* region, int W, int H, int R,
                       const orc_ransac_params* prm, const double* eps, int32_t* npts, int32_t* triples,
                       double* planes, uint8_t* hvalid, double* errors, int32_t* counts, int32_t* counts_lo,
                       int32_t* counts_hi, int32_t* jstar, uint8_t* stored, double* centroids, int8_t* labels) {
    size_t n = (size_t)W * H;
    const int nh = prm->hyps;
    int32_t* list = (int32_t*)malloc((n > 0 ? n : 1) * sizeof(int32_t));
    for (size_t p = 0; p < n; ++p) labels[p] = -1;
    int n_stored = 0;
    for (int g = 0; g < R; ++g) {
        int m = 0;
        for (size_t p = 0; p < n; ++p)
            if ((valid[p] & 1) && region[p] == g) list[m++] = (int32_t)p;
        npts[g] = m;
        int32_t* tr = triples + (size_t)g * nh * 3;
        double* pls = planes + (size_t)g * nh * 4;
        uint8_t* hv = hvalid + (size_t)g * nh;
#pragma omp parallel for schedule(static)
        for (int j = 0; j < nh; ++j) {
            int slot[3] = {-1, -1, -1};
            int got = 0;
            for (int b = 0; b < 16 && got < 3 && m > 0; ++b) {
                uint64_t ctr[4] = {(uint64_t)j, (uint64_t)g, (uint64_t)b, 1};
                uint64_t key[2] = {prm->seed, prm->frame};
                uint64_t w[4];
                orc_philox4x64_10(ctr, key, w);
                for (int q = 0; q < 4 && got < 3; ++q) {
                    int k = (int)(((unsigned __int128)w[q] * (uint64_t)m) >> 64);
                    int dup = 0;
                    for (int s = 0; s < got; ++s)
                        if (slot[s] == k) dup = 1;
                    if (!dup) slot[got++] = k;
                }
            }
            double* pl = pls + 4 * (size_t)j;
            pl[0] = pl[1] = pl[2] = pl[3] = 0.0;
            hv[j] = 0;
            for (int s = 0; s < 3; ++s) tr[3 * j + s] = got == 3 ? slot[s] : -1;
            if (got < 3) continue;
            double p0[3], p1[3], p2[3];
            point_at(P, n, list[slot[0]], p0);
            point_at(P, n, list[slot[1]], p1);
            point_at(P, n, list[slot[2]], p2);
            double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
            double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
            double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                           e1[0] * e2[1] - e1[1] * e2[0]};
            double cn = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
            double l2 = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
            if (!(cn > 1e-3 * l1 * l2)) continue;
            double nn[3] = {c[0] / cn, c[1] / cn, c[2] / cn};
            double d = -(nn[0] * p0[0] + nn[1] * p0[1] + nn[2] * p0[2]);
            if (d < 0) {
                nn[0] = -nn[0]; nn[1] = -nn[1]; nn[2] = -nn[2];
                d = -d;
            }
            pl[0] = nn[0]; pl[1] = nn[1]; pl[2] = nn[2]; pl[3] = d;
            hv[j] = 1;
        }
        /* Alg. 2 inner loop over every point of the region */
#pragma omp parallel for schedule(dynamic, 4)
        for (int j = 0; j < nh; ++j) {
            size_t o = (size_t)g * nh + j;
            double e = 0.0;
            int32_t c = 0, clo = 0, chi = 0;
            if (hv[j]) {
                const double* pl = pls + 4 * (size_t)j;
                double tlo = eps ? prm->thresh - eps[o] : prm->thresh;
                double thi = eps ? prm->thresh + eps[o] : prm->thresh;
                for (int i = 0; i < m; ++i) {
                    double p[3];
                    point_at(P, n, list[i], p);
                    double dist = fabs(pl[0] * p[0] + pl[1] * p[1] + pl[2] * p[2] + pl[3]);
                    e += dist;
                    c += dist < prm->thresh;
                    clo += dist < tlo;
                    chi += dist < thi;
                }
            }
            errors[o] = hv[j] ? e : INFINITY;
            counts[o] = c;
            if (counts_lo) counts_lo[o] = clo;
            if (counts_hi) counts_hi[o] = chi;
        }
        int best = -1;
        double best_err = INFINITY;
        for (int j = 0; j < nh; ++j)
            if (hv[j] && errors[(size_t)g * nh + j] < best_err) {
                best_err = errors[(size_t)g * nh + j];
                best = j;
            }
        jstar[g] = best;
        stored[g] = best >= 0 && 10LL * counts[(size_t)g * nh + best] > 9LL * m;
        double* ce = centroids + 3 * (size_t)g;
        ce[0] = ce[1] = ce[2] = 0.0;
        if (!stored[g]) continue;
        ++n_stored;
        const double* pl = pls + 4 * (size_t)best;
        double s[3] = {0.0, 0.0, 0.0};
        int cnt = 0;
        for (int i = 0; i < m; ++i) {
            double p[3];
            point_at(P, n, list[i], p);
            if (fabs(pl[0] * p[0] + pl[1] * p[1] + pl[2] * p[2] + pl[3]) < prm->thresh) {
                labels[list[i]] = (int8_t)g;
                s[0] += p[0]; s[1] += p[1]; s[2] += p[2];
                ++cnt;
            }
        }
        ce[0] = s[0] / cnt; ce[1] = s[1] / cnt; ce[2] = s[2] / cnt;
    }
    free(list);
    return n_stored;
}

/* ------------------------------------------------------------------------ */
/* Segmentation of the normal image (Sec. III-D: Canny edges on the normal   */
/* image; the regions between edges are the candidate planes).              */
/* The paper names the steps only; the readings:                            */
/*  - gradient of the vector image: 3x3 Sobel sums of each normal channel   */
/*    (the kernels of Eq. 2), structure tensor Exx = sum gx^2, Eyy = sum     */
/*    gy^2, Exy = sum gx gy; magnitude^2 m2 = Exx + Eyy; edge direction      */
/*    from the doubled angle (A, B) = (Exx - Eyy, 2 Exy) of the principal    */
/*    eigenvector, in four sectors;                                          */
/*  - a pixel whose 3x3 window holds an invalid normal is a barrier (no     */
/*    gradient, no edge, no region);                                         */
/*  - non-maximum suppression along the sector: keep m2 > m2(behind) and     */
/*    m2 >= m2(ahead); thresholds m2 > low^2 (weak), m2 > high^2 (strong);    */
/*    hysteresis keeps weak pixels 8-connected to a strong one;              */
/*  - regions: 4-connected components of valid, non-barrier pixels with no   */
/*    edge pixel in their 3x3 window (edges closed by one dilation), with at */
/*    least min_area pixels, numbered by size (ties: smallest pixel index    */
/*    first), at most max_regions.                                           */
/* All floating-point decisions are taken in FP32 (float, no contraction),  */
/* in the order written here.                                               */
/* ------------------------------------------------------------------------ */
void orc_seg_grad(const float* N, const uint8_t* nvalid, int W, int H, float* m2, uint8_t* sector, uint8_t* barrier) {
    const size_t n = (size_t)W * H;
#pragma omp parallel for schedule(static)
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            int ok = u >= 1 && u < W - 1 && v >= 1 && v < H - 1;
            for (int dv = -1; dv <= 1 && ok; ++dv)
                for (int du = -1; du <= 1; ++du)
                    if (!nvalid[p + (ptrdiff_t)dv * W + du]) ok = 0;
            barrier[p] = !ok;
            m2[p] = 0.0f;
            sector[p] = 0;
            if (!ok) continue;
            float exx = 0.0f, eyy = 0.0f, exy = 0.0f;
            for (int c = 0; c < 3; ++c) {
                const float* ch = N + (size_t)c * n;
#define NV(du, dv) ch[p + (ptrdiff_t)(dv) * W + (du)]
                /* Sobel sums: right minus left column (1,2,1 rows); bottom minus top row */
                float gx = ((NV(1, -1) - NV(-1, -1)) + 2.0f * (NV(1, 0) - NV(-1, 0))) + (NV(1, 1) - NV(-1, 1));
                float gy = ((NV(-1, 1) - NV(-1, -1)) + 2.0f * (NV(0, 1) - NV(0, -1))) + (NV(1, 1) - NV(1, -1));
#undef NV
                exx = exx + gx * gx;
                eyy = eyy + gy * gy;
                exy = exy + gx * gy;
            }
            m2[p] = exx + eyy;
            float A = exx - eyy, B = 2.0f * exy;
            /* sector of theta = atan2(B, A) / 2: 0 across columns, 1 along (+1,+1), 2 across rows, 3 along (+1,-1) */
            float aA = fabsf(A), aB = fabsf(B);
            uint8_t s;
            if (aB <= aA) s = A >= 0.0f ? 0 : 2;
            else s = B > 0.0f ? 1 : 3;
            sector[p] = s;
        }
}

static const int SEC_DU[4] = {1, 1, 0, 1};
static const int SEC_DV[4] = {0, 1, 1, -1};

void orc_seg_edges(const float* m2, const uint8_t* sector, const uint8_t* barrier, int W, int H, float low, float high,
                   uint8_t* cls, uint8_t* edge) {
    const size_t n = (size_t)W * H;
    const float lo2 = low * low, hi2 = high * high;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            cls[p] = 0;
            if (barrier[p]) continue;
            int s = sector[p];
            int ua = u + SEC_DU[s], va = v + SEC_DV[s], ub = u - SEC_DU[s], vb = v - SEC_DV[s];
            float ahead = (ua >= 0 && ua < W && va >= 0 && va < H) ? m2[(size_t)va * W + ua] : 0.0f;
            float behind = (ub >= 0 && ub < W && vb >= 0 && vb < H) ? m2[(size_t)vb * W + ub] : 0.0f;
            if (!(m2[p] > behind && m2[p] >= ahead)) continue;
            cls[p] = m2[p] > hi2 ? 2 : (m2[p] > lo2 ? 1 : 0);
        }
    /* hysteresis: breadth-first from every strong pixel through weak ones (8-connectivity) */
    int32_t* q = (int32_t*)malloc((n > 0 ? n : 1) * sizeof(int32_t));
    for (size_t p = 0; p < n; ++p) edge[p] = 0;
    size_t head = 0, tail = 0;
    for (size_t p = 0; p < n; ++p)
        if (cls[p] == 2) {
            edge[p] = 1;
            q[tail++] = (int32_t)p;
        }
    while (head < tail) {
        int p = q[head++];
        int u = p % W, v = p / W;
        for (int dv = -1; dv <= 1; ++dv)
            for (int du = -1; du <= 1; ++du) {
                int uu = u + du, vv = v + dv;
                if (uu < 0 || uu >= W || vv < 0 || vv >= H) continue;
                size_t qq = (size_t)vv * W + uu;
                if (cls[qq] >= 1 && !edge[qq]) {
                    edge[qq] = 1;
                    q[tail++] = (int32_t)qq;
                }
            }
    }
    free(q);
}

typedef struct {
    int32_t size, root;
} seg_comp;

static int seg_comp_cmp(const void* a, const void* b) {
    const seg_comp* x = (const seg_comp*)a;
    const seg_comp* y = (const seg_comp*)b;
    if (x->size != y->size) return x->size > y->size ? -1 : 1;
    return x->root < y->root ? -1 : (x->root > y->root);
}

/* region pixels: mask != 0; 4-connected components (breadth-first), ranked. Returns the number of regions. */
int orc_seg_regions(const uint8_t* mask, int W, int H, int min_area, int max_regions, int16_t* region) {
    const size_t n = (size_t)W * H;
    int32_t* comp = (int32_t*)malloc((n > 0 ? n : 1) * sizeof(int32_t));
    int32_t* q = (int32_t*)malloc((n > 0 ? n : 1) * sizeof(int32_t));
    seg_comp* cs = (seg_comp*)malloc((n > 0 ? n : 1) * sizeof(seg_comp));
    int nc = 0;
    for (size_t p = 0; p < n; ++p) comp[p] = -1;
    for (size_t p0 = 0; p0 < n; ++p0) {
        if (!mask[p0] || comp[p0] >= 0) continue;
        size_t head = 0, tail = 0;
        q[tail++] = (int32_t)p0;
        comp[p0] = nc;
        while (head < tail) {
            int p = q[head++];
            int u = p % W, v = p / W;
            const int du[4] = {1, -1, 0, 0}, dv[4] = {0, 0, 1, -1};
            for (int k = 0; k < 4; ++k) {
                int uu = u + du[k], vv = v + dv[k];
                if (uu < 0 || uu >= W || vv < 0 || vv >= H) continue;
                size_t qq = (size_t)vv * W + uu;
                if (mask[qq] && comp[qq] < 0) {
                    comp[qq] = nc;
                    q[tail++] = (int32_t)qq;
                }
            }
        }
        cs[nc].size = (int32_t)tail;
        cs[nc].root = (int32_t)p0; /* the first pixel met in row-major order is the smallest index */
        ++nc;
    }
    int32_t* rank = (int32_t*)malloc((nc > 0 ? nc : 1) * sizeof(int32_t));
    seg_comp* sorted = (seg_comp*)malloc((nc > 0 ? nc : 1) * sizeof(seg_comp));
    memcpy(sorted, cs, (size_t)nc * sizeof(seg_comp));
    qsort(sorted, (size_t)nc, sizeof(seg_comp), seg_comp_cmp);
    for (int i = 0; i < nc; ++i) rank[i] = -1;
    int nr = 0;
    for (int i = 0; i < nc && nr < max_regions; ++i) {
        if (sorted[i].size < min_area) break;
        rank[comp[sorted[i].root]] = nr++;
    }
    for (size_t p = 0; p < n; ++p) region[p] = (int16_t)(comp[p] >= 0 ? rank[comp[p]] : -1);
    free(comp); free(q); free(cs); free(rank); free(sorted);
    return nr;
}

/* The whole segmentation: gradient, edges, regions of valid-normal, non-barrier, non-edge pixels. */
int orc_segment(const float* N, const uint8_t* nvalid, int W, int H, float low, float high, int min_area,
                int max_regions, int16_t* region, uint8_t* edge_out) {
    const size_t n = (size_t)W * H;
    float* m2 = (float*)malloc((n > 0 ? n : 1) * sizeof(float));
    uint8_t* sec = (uint8_t*)malloc(n > 0 ? n : 1);
    uint8_t* bar = (uint8_t*)malloc(n > 0 ? n : 1);
    uint8_t* cls = (uint8_t*)malloc(n > 0 ? n : 1);
    uint8_t* edge = (uint8_t*)malloc(n > 0 ? n : 1);
    orc_seg_grad(N, nvalid, W, H, m2, sec, bar);
    orc_seg_edges(m2, sec, bar, W, H, low, high, cls, edge);
    /* region pixels: valid, no barrier, no edge pixel in the 3x3 window (the
       edges closed by one dilation, which seals the gaps suppression leaves
       where three planes meet) */
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            int near_edge = 0;
            for (int dv = -1; dv <= 1; ++dv)
                for (int du = -1; du <= 1; ++du) {
                    int uu = u + du, vv = v + dv;
                    if (uu >= 0 && uu < W && vv >= 0 && vv < H && edge[(size_t)vv * W + uu]) near_edge = 1;
                }
            cls[p] = nvalid[p] && !bar[p] && !near_edge;
        }
    int nr = orc_seg_regions(cls, W, H, min_area, max_regions, region);
    if (edge_out) memcpy(edge_out, edge, n);
    free(m2); free(sec); free(bar); free(cls); free(edge);
    return nr;
}

/* ------------------------------------------------------------------------ */
/* Region contours simplified into polygons (Sec. III-D: contours of the     */
/* segmented normal image, simplified into polygons).  Readings:            */
/*  - the contour of region g is its outer boundary, traced with the Moore  */
/*    neighbourhood clockwise (on screen, y down) from the region's first   */
/*    pixel in row-major order, entered from the west; the trace stops when */
/*    it is back on the first pixel and would repeat its first move;        */
/*  - simplification: Douglas-Peucker on the closed contour, split at the   */
/*    contour point farthest from the first (the first such in order); a    */
/*    point is kept iff its distance to the current chord exceeds eps px;   */
/*  - vertices are pixel coordinates (x = column, y = row), clockwise from  */
/*    the first pixel.                                                      */
/* ------------------------------------------------------------------------ */
static const int MOORE_DX[8] = {-1, -1, 0, 1, 1, 1, 0, -1}; /* W NW N NE E SE S SW */
static const int MOORE_DY[8] = {0, -1, -1, -1, 0, 1, 1, 1};

static int in_region(const int16_t* reg, int W, int H, int x, int y, int g) {
    return x >= 0 && x < W && y >= 0 && y < H && reg[(size_t)y * W + x] == g;
}

/* Boundary pixels of region g from its first pixel (sx, sy), into bx/by
 * (capacity cap, at least 4 n_g + 8); returns their number.  b is the
 * direction from the current pixel to the last outside pixel checked.  The
 * trace ends when it stands on the start pixel again and its next move
 * would repeat the first move out of it. */
static int trace_boundary(const int16_t* reg, int W, int H, int g, int sx, int sy, int* bx, int* by, int cap) {
    int n = 0, cx = sx, cy = sy, b = 0; /* entered from the west */
    int fx = -1, fy = -1;               /* the first move's target */
    bx[n] = sx; by[n] = sy; ++n;
    for (int guard = 0; guard < cap; ++guard) {
        int found = -1;
        for (int k = 1; k <= 8; ++k) {
            int d = (b + k) & 7;
            if (in_region(reg, W, H, cx + MOORE_DX[d], cy + MOORE_DY[d], g)) { found = d; break; }
        }
        if (found < 0) break; /* a single pixel */
        int ox = cx + MOORE_DX[(found + 7) & 7], oy = cy + MOORE_DY[(found + 7) & 7];
        int nx = cx + MOORE_DX[found], ny = cy + MOORE_DY[found];
        if (guard == 0) { fx = nx; fy = ny; }
        else if (cx == sx && cy == sy && nx == fx && ny == fy) { --n; break; } /* drop the repeated start */
        int nb = 0;
        for (int d = 0; d < 8; ++d)
            if (nx + MOORE_DX[d] == ox && ny + MOORE_DY[d] == oy) nb = d;
        if (n >= cap) break;
        bx[n] = nx; by[n] = ny; ++n;
        cx = nx; cy = ny; b = nb;
    }
    return n;
}

/* distance of p to the line through a and c (to a when a == c) */
static double chord_dist(double px, double py, double ax, double ay, double cx, double cy) {
    double dx = cx - ax, dy = cy - ay;
    double len = sqrt(dx * dx + dy * dy);
    if (len == 0.0) return sqrt((px - ax) * (px - ax) + (py - ay) * (py - ay));
    return fabs(dx * (py - ay) - dy * (px - ax)) / len;
}

/* Douglas-Peucker on the open chain idx[0..m-1] of points (bx, by): keep[] marks kept ones */
static void dp_chain(const int* bx, const int* by, const int* idx, int m, double eps, uint8_t* keep, int* stack) {
    keep[0] = keep[m - 1] = 1;
    int top = 0;
    stack[top++] = 0; stack[top++] = m - 1;
    while (top > 0) {
        int hi = stack[--top], lo = stack[--top];
        if (hi - lo < 2) continue;
        double best = -1.0;
        int bi = -1;
        for (int i = lo + 1; i < hi; ++i) {
            double d = chord_dist(bx[idx[i]], by[idx[i]], bx[idx[lo]], by[idx[lo]], bx[idx[hi]], by[idx[hi]]);
            if (d > best) { best = d; bi = i; }
        }
        if (best > eps) {
            keep[bi] = 1;
            stack[top++] = lo; stack[top++] = bi;
            stack[top++] = bi; stack[top++] = hi;
        }
    }
}

int orc_region_polygons(const int16_t* region, int W, int H, int n_regions, double eps, int32_t* xy,
                        int max_vertices, int32_t* offsets) {
    const size_t n = (size_t)W * H;
    int cap = 4 * (int)n + 8;
    int* bx = (int*)malloc((size_t)cap * sizeof(int));
    int* by = (int*)malloc((size_t)cap * sizeof(int));
    int* idx = (int*)malloc((size_t)(cap + 1) * sizeof(int));
    int* stack = (int*)malloc((size_t)(2 * cap + 8) * sizeof(int));
    uint8_t* keep = (uint8_t*)malloc((size_t)cap + 1);
    int total = 0;
    for (int g = 0; g < n_regions; ++g) {
        offsets[g] = total;
        size_t first = n;
        for (size_t p = 0; p < n; ++p)
            if (region[p] == g) { first = p; break; }
        if (first == n) continue;
        int sx = (int)(first % W), sy = (int)(first / W);
        int m = trace_boundary(region, W, H, g, sx, sy, bx, by, cap);
        int kept_n = 0;
        int* out_i = idx; /* reuse: indices of the kept points, in contour order */
        if (m <= 2) {
            for (int i = 0; i < m; ++i) out_i[kept_n++] = i;
        } else {
            int far = 0;
            double fd = -1.0;
            for (int i = 1; i < m; ++i) {
                double d = sqrt((double)(bx[i] - sx) * (bx[i] - sx) + (double)(by[i] - sy) * (by[i] - sy));
                if (d > fd) { fd = d; far = i; }
            }
            /* chain A = 0..far, chain B = far..m-1, 0 */
            int* ca = (int*)malloc((size_t)(m + 1) * sizeof(int));
            uint8_t* ka = (uint8_t*)calloc((size_t)m + 1, 1);
            for (int i = 0; i <= far; ++i) ca[i] = i;
            dp_chain(bx, by, ca, far + 1, eps, ka, stack);
            for (int i = 0; i < far; ++i)
                if (ka[i]) out_i[kept_n++] = ca[i];
            int mb = m - far + 1;
            for (int i = 0; i < mb; ++i) ca[i] = i < m - far ? far + i : 0;
            memset(ka, 0, (size_t)m + 1);
            dp_chain(bx, by, ca, mb, eps, ka, stack);
            for (int i = 0; i < mb - 1; ++i)
                if (ka[i]) out_i[kept_n++] = ca[i];
            free(ca);
            free(ka);
        }
        for (int i = 0; i < kept_n; ++i) {
            if (total < max_vertices) {
                xy[2 * total] = bx[out_i[i]];
                xy[2 * total + 1] = by[out_i[i]];
            }
            ++total;
        }
    }
    offsets[n_regions] = total;
    free(bx); free(by); free(idx); free(stack); free(keep);
    return total;
}
