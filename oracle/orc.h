/*
 * CPU FP64 oracle of the plane-extraction path.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never
 * does.  It shares no code, header, table or helper with the GPU library.
 *
 * Every function follows a passage of arXiv 2411.01919 ("Real-Time Polygonal
 * Semantic Mapping for Humanoid Robot Stair Climbing"), cited per function,
 * with the readings of the paper listed beside each.
 *
 * Units: depth in millimetres (uint16, 0 = hole), diffusion in millimetres,
 * points / planes / thresholds in metres.  Images are row-major [H][W];
 * 3-vectors per pixel are stored as planes [3][H][W].
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Perona-Malik diffusion, Eq. 1 / Alg. 1, of a depth image in mm (a pixel is a
 * hole iff its input value is not > 0; uint16 frames are passed converted).
 * edge_stop 0: g = exp(-(x/k)^2), 1: g = 1/(1+(x/k)^2).
 * out: float64 [H][W] mm, holes stay 0. */
void orc_diffuse(const double* depth, int W, int H, int iters, double lambda, double kappa,
                 int edge_stop, double* out);

/* Diffusion variants: scheme 1 = Alg. 1 as printed (pixel-centred c_p lap I),
 * scheme 2 = 8-neighbour per-edge flux (diagonals weight 1/2, distance sqrt 2). */
void orc_diffuse_variant(const double* depth, int W, int H, int iters, double lambda, double kappa,
                         int edge_stop, int scheme, double* out);

/* Back-projection (Sec. III-D, Alg. 2): P [3][H][W] metres, valid [H][W] (1 = depth > 0). */
void orc_backproject(const double* depth_mm, int W, int H, double fx, double fy, double cx, double cy,
                     double* P, uint8_t* valid);

/* Normal image (Eq. 2 / Alg. 1, reading: Sobel of the point image, n = -(Gx x Gy)/|.|).
 * N [3][H][W]; nvalid [H][W]; gx, gy optional ([3][H][W]) Sobel sums for conditioning checks. */
void orc_normals(const double* P, const uint8_t* valid, int W, int H, double* N, uint8_t* nvalid,
                 double* gx, double* gy);

/* Row-major list of depth-valid pixel indices; returns M0. */
int orc_valid_list(const uint8_t* valid, int npx, int32_t* L);

typedef struct {
    int hyps;            /* hypotheses per round */
    int max_planes;      /* rounds */
    int min_inliers;     /* emit iff |F| >= min_inliers */
    double thresh;       /* inlier threshold t (m), strict < */
    uint64_t seed;       /* Philox key word 0 */
    uint64_t frame;      /* Philox key word 1 */
} orc_ransac_params;

/* Hypotheses of round r (Alg. 2: select 3 random points, fit a plane).
 * assigned[px] != 0 marks pixels removed by earlier rounds.
 * triples [hyps][3] (positions in L), planes [hyps][4] (n, d), hvalid [hyps]. */
void orc_hypotheses(const double* P, int W, int H, const int32_t* L, int M0, const uint8_t* assigned,
                    const orc_ransac_params* prm, int r, int32_t* triples, double* planes, uint8_t* hvalid);

/* Inlier counts (Alg. 2 inner loop, Eq. 3 distance) over the unassigned valid
 * points of L.  counts[j] = #{|n.p + d| < t}; when eps != NULL also
 * counts_lo[j] = #{|r| < t - eps[j]} and counts_hi[j] = #{|r| < t + eps[j]}.
 * Invalid hypotheses score 0.  If pmax != NULL it receives max |p| over the set. */
void orc_score(const double* P, int W, int H, const int32_t* L, int M0, const uint8_t* assigned,
               const double* planes, const uint8_t* hvalid, int nh, double thresh, const double* eps,
               int32_t* counts, int32_t* counts_lo, int32_t* counts_hi, double* pmax);

/* Total-least-squares plane of the points P[idx[0..n-1]] (smallest-eigenvalue
 * eigenvector of the scatter about the centroid), camera-facing: d >= 0.
 * plane[4] = (n, d), centroid[3].  Returns 0, or -1 if n < 3. */
int orc_refit(const double* P, int W, int H, const int32_t* idx, int n, double plane[4], double centroid[3]);

/* Symmetric 3x3 eigen-decomposition by cyclic Jacobi: A (row-major, symmetric)
 * -> eigenvalues w[3] ascending, eigenvectors as columns of V (row-major). */
void orc_eig3(const double A[9], double w[3], double V[9]);

typedef struct {
    int status;          /* 0 emitted; 1 no valid hypothesis; 2 |F| < min_inliers; 3 < 3 points left */
    int jstar;
    int n_remaining;     /* |R_r| before this round */
    int s_count;         /* |S| = inliers of the hypothesis j* */
    int f_count;         /* |F| */
    double hyp_plane[4]; /* plane of j* */
    double plane[4];     /* refit plane */
    double centroid[3];
} orc_round_result;

/* One round of sequential RANSAC given the assignment state (follow mode).
 * Outputs per-hypothesis data (any may be NULL), S/F masks over pixels
 * (smask/fmask [H][W], 1 = member; may be NULL). */
void orc_ransac_round(const double* P, int W, int H, const int32_t* L, int M0, const uint8_t* assigned,
                      const orc_ransac_params* prm, int r, const double* eps,
                      int32_t* triples, double* planes, uint8_t* hvalid,
                      int32_t* counts, int32_t* counts_lo, int32_t* counts_hi,
                      uint8_t* smask, uint8_t* fmask, orc_round_result* res);

/* Region-mode RANSAC, Alg. 2 as printed: for each region label g in [0, R)
 * (other labels and depth holes belong to no region), hyps hypotheses drawn
 * from the region's row-major point list with counter (j, g, b, 1); the model
 * with the smallest sum of |n.p + d| over the region (ties to the smaller j)
 * is stored iff 10 inliers > 9 n_g.  Arrays: npts [R]; triples [R][hyps][3]
 * (list positions, -1 when fewer than 3 were drawn); planes [R][hyps][4];
 * hvalid, errors (INFINITY without a plane), counts [R][hyps]; with eps
 * [R][hyps] also counts_lo/hi at t -/+ eps; jstar [R] (-1 none); stored [R];
 * centroids [R][3]; labels [H][W] int8.  Returns the number stored. */
int orc_ransac_regions(const double* P, const uint8_t* valid, const int16_t* region, int W, int H, int R,
                       const orc_ransac_params* prm, const double* eps, int32_t* npts, int32_t* triples,
                       double* planes, uint8_t* hvalid, double* errors, int32_t* counts, int32_t* counts_lo,
                       int32_t* counts_hi, int32_t* jstar, uint8_t* stored, double* centroids, int8_t* labels);

/* Segmentation of the normal image (Canny edges, then regions).  N [3][H][W]
 * FP32 normals, nvalid [H][W].  Every floating-point decision is in FP32.
 * orc_seg_grad: m2 = Exx + Eyy of the channels' Sobel sums, sector 0..3 of
 * the edge normal, barrier = an invalid normal in the 3x3 window.
 * orc_seg_edges: cls 0/1 weak/2 strong after non-maximum suppression, edge =
 * hysteresis result.  orc_seg_regions: ranked 4-connected components of
 * mask.  orc_segment: all of it; returns the number of regions. */
void orc_seg_grad(const float* N, const uint8_t* nvalid, int W, int H, float* m2, uint8_t* sector, uint8_t* barrier);
void orc_seg_edges(const float* m2, const uint8_t* sector, const uint8_t* barrier, int W, int H, float low, float high,
                   uint8_t* cls, uint8_t* edge);
int orc_seg_regions(const uint8_t* mask, int W, int H, int min_area, int max_regions, int16_t* region);
int orc_segment(const float* N, const uint8_t* nvalid, int W, int H, float low, float high, int min_area,
                int max_regions, int16_t* region, uint8_t* edge_out);

/* Contours of the regions 0..n_regions-1 of a label image, simplified into
 * polygons (Moore tracing clockwise from each region's first pixel, Jacob's
 * stop; Douglas-Peucker with tolerance eps px on the closed contour).
 * xy [max_vertices][2] (x, y) pixel vertices; offsets [n_regions+1].
 * Returns the total vertex count (may exceed max_vertices: nothing past it
 * is written). */
int orc_region_polygons(const int16_t* region, int W, int H, int n_regions, double eps, int32_t* xy,
                        int max_vertices, int32_t* offsets);

/* Whole-frame sequential RANSAC.  labels [H][W] int8 (-1 none), planes_out
 * [max_planes][4], centroids_out [max_planes][3], inliers_out, jstar_out
 * [max_planes] (NULL allowed).  Returns the number of planes emitted;
 * *residuals receives sum_r |R_r| * hyps over the rounds that scored. */
int orc_ransac(const double* P, const uint8_t* valid, int W, int H, const orc_ransac_params* prm,
               int8_t* labels, double* planes_out, double* centroids_out, int32_t* inliers_out,
               int32_t* jstar_out, double* residuals);

/* Number of OpenMP threads the oracle uses (for the benchmark record). */
int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
