/*
 * pp.h -- C ABI of the MI355X (gfx950) plane-extraction library libpp.so.
 *
 * The library computes the per-frame plane-extraction path of "Real-Time
 * Polygonal Semantic Mapping for Humanoid Robot Stair Climbing"
 * (arXiv 2411.01919):
 *   1. Perona-Malik anisotropic diffusion of a depth image (Sec. III-C, Eq. 1,
 *      Alg. 1),
 *   2. back-projection of the depth image to a point image with the camera
 *      intrinsics (Sec. III-D, Alg. 2),
 *   3. the normal image from Sobel gradients (Sec. III-C, Eq. 2, Alg. 1),
 *   4. RANSAC plane extraction: random 3-point hypotheses, inlier scoring with
 *      the point-to-plane distance (Eq. 3, Alg. 2), selection, a
 *      least-squares refit of the winning plane (the best plane model of
 *      Sec. III-A) and removal of its inliers, repeated for up to
 *      max_planes planes per frame.
 * Every stage runs as hand-written HIP kernels on the GPU.
 *
 * Conventions (all calls):
 *  - Plain C types only.  Every pointer named *_dev is a device pointer the
 *    caller allocated and owns; the library never frees caller memory.
 *  - Images are row-major with a row pitch in pixels (pitch_px >= width);
 *    3-vector images are three planes [3][height][pitch_px].
 *  - Depth is uint16 millimetres with 0 = hole; diffused depth is float mm;
 *    points, planes and thresholds are in metres; camera frame x right,
 *    y down, z forward; pixel (u, v) = (column, row) looks along
 *    ((u - cx)/fx, (v - cy)/fy, 1).
 *  - hip_stream is a hipStream_t (NULL = the null stream).  Calls enqueue
 *    their kernels asynchronously and return; outputs are valid once the
 *    stream has reached that point.  Counts the host needs (number of
 *    planes) are written to device memory, so no call synchronises.
 *  - Arguments are checked before any HIP call; a bad argument returns
 *    PP_E_INVAL and enqueues nothing.  A failing HIP call returns PP_E_HIP and
 *    poisons the context: every later call on it returns PP_E_HIP until it is
 *    destroyed.  pp_last_error() describes the last failure.
 *  - A pp_ctx is not thread-safe; use one per thread (or serialise).  It owns
 *    scratch memory that grows to the largest shape seen and is reused.  Its
 *    calls may use different streams: a call on a stream other than the
 *    previous call's first waits (on the device) for the previous call's
 *    work, since both use the context's frame tables and scratch; work on
 *    one context therefore runs in call order.  A stream under the caller's
 *    graph capture is not ordered this way: the caller orders its graph.
 *    Graphs captured by pp_batch_run are kept per batch layout, at most 64
 *    (the least recently used is destroyed once its last launch is done).
 */
#ifndef PP_H
#define PP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pp_status;
enum {
    PP_OK = 0,
    PP_PENDING = 1,         /* pp_poll: result not ready yet */
    PP_E_INVAL = -1,        /* bad argument (nothing was enqueued) */
    PP_E_NOMEM = -2,        /* device allocation failed */
    PP_E_BUDGET = -3,       /* a frame can never fit the server's HBM budget */
    PP_E_HIP = -4,          /* a HIP runtime call failed; the object is poisoned */
    PP_E_NODEVICE = -5,     /* no usable GPU */
    PP_E_CLOSED = -6,       /* server/stream closed or destroyed */
    PP_E_UNSUPPORTED = -7,  /* valid request outside what this library implements */
    PP_E_TIMEOUT = -8,      /* reserved */
    PP_E_AGAIN = -9         /* pp_submit: the stream's staging is full; poll results, then retry */
};

typedef struct pp_ctx pp_ctx;

typedef struct { float fx, fy, cx, cy; } pp_intrinsics;              /* pixels */
typedef struct { int32_t width, height, pitch_px; } pp_frame_desc;   /* 3 <= w,h <= 16384; w*h <= 2^27 */

enum { PP_EDGE_EXP = 0, PP_EDGE_RATIONAL = 1 };
/* Discretisations of Eq. 1:
 *  PP_DIFFUSE_EDGE4  per-edge flux over the 4-neighbourhood,
 *                    I_p += lambda sum_q g(|I_q - I_p|) (I_q - I_p): conservative,
 *                    zero flux into holes and across the border (the default);
 *  PP_DIFFUSE_PIXEL  Alg. 1 as printed: c_p = g(|grad I_p|), the gradient from
 *                    central differences (one-sided beside a hole or the border),
 *                    I_p += lambda c_p sum_q (I_q - I_p) over valid 4-neighbours;
 *  PP_DIFFUSE_EDGE8  per-edge flux over the 8-neighbourhood, diagonal edges at
 *                    distance sqrt 2 with weight 1/2: I_p += lambda sum_q w_q
 *                    g(|I_q - I_p| / d_q) (I_q - I_p). */
enum { PP_DIFFUSE_EDGE4 = 0, PP_DIFFUSE_PIXEL = 1, PP_DIFFUSE_EDGE8 = 2 };
/* Alg. 1 parameters: iterations N, step gamma (lambda), edge scale k (kappa, mm).
 * edge_stop PP_EDGE_EXP: g(x) = exp(-(x/kappa)^2) as Alg. 1 prints it;
 * PP_EDGE_RATIONAL: g(x) = 1/(1 + (x/kappa)^2) (Perona and Malik's second
 * function).  kappa > 0; 0 < lambda <= 0.25 (EDGE4, PIXEL) or <= 1/6 (EDGE8),
 * the bounds under which every step is a convex combination of neighbours. */
typedef struct { int32_t iters; float lambda; float kappa_mm; int32_t edge_stop; int32_t scheme; } pp_diffuse_params;

/* Inlier scoring arithmetic.  Every form decides |n.p + d| < t exactly as the
 * canonical FP32 residual fmaf(nx,x, fmaf(ny,y, fmaf(nz,z,d))) does, so all
 * forms return identical counts, planes and labels:
 *  PP_SCORE_FP32      the canonical formula on the vector ALUs;
 *  the matrix-core forms evaluate on the matrix cores the points of the
 *  64-point tiles whose bounding box leaves a hypothesis undecided (when a
 *  tile has at least 40 such hypotheses; fewer go to the vector ALUs):
 *  PP_SCORE_MFMA_F32  the contraction in FP32; residuals within
 *                     max(recheck_band_m, 16 * 2^-24 * (max|p|_1 + |d|)) of t
 *                     are recomputed canonically;
 *  PP_SCORE_BF16/FP16 points centred on their tile's box and the normals in
 *                     BF16/FP16, FP32 accumulation; residuals within
 *                     max(recheck_band_m, a bound on the low-precision
 *                     error, about 1e-2 / 1e-3 of the tile's extent along n)
 *                     of t are recomputed canonically (recheck_band_m =
 *                     0.002 is the 2 mm form, 0 the tightest). */
enum { PP_SCORE_FP32 = 0, PP_SCORE_MFMA_F32 = 1, PP_SCORE_BF16 = 2, PP_SCORE_FP16 = 3 };

/* Alg. 2 "RANSAC parameters".  Hypotheses draw from Philox4x64-10 keyed by
 * (seed, frame_id) with counter (hypothesis, round, block, 0).
 * 1 <= max_planes <= 127; 1 <= hyps_per_plane <= 8192; thresh_m > 0;
 * min_inliers >= 1; recheck_band_m >= 0 (used by the MFMA forms). */
typedef struct {
    int32_t max_planes;
    int32_t hyps_per_plane;
    int32_t min_inliers;
    float thresh_m;
    uint64_t seed;
    uint64_t frame_id;
    int32_t precision;      /* PP_SCORE_* */
    float recheck_band_m;
} pp_ransac_params;

/* One extracted plane: n.p + d = 0 with |n| = 1 and d >= 0 (faces the camera). */
typedef struct {
    double n[3];
    double d;
    double centroid[3];
    int32_t inliers;        /* |F|: points labelled with this plane */
    int32_t hyp_index;      /* winning hypothesis j* of the round */
} pp_plane;

/* Optional introspection of pp_ransac_planes (any pointer may be NULL).
 * Device buffers, caller-owned; masks must be zeroed by the caller.
 * counts [max_planes][hyps], hyps [max_planes][hyps][4] (n, d; d = NaN when
 * invalid), triples [max_planes][hyps][3] (positions in the valid list, -1
 * when sampling gave up), round_info [max_planes][4] = (j*, |S|, |F|, status:
 * 0 plane emitted, 1 no valid hypothesis, 2 |F| < min_inliers, -1 not run),
 * masks [max_planes][height*width] (bit0: inlier of j*, bit1: in F),
 * valid_list [height*width] (pixel offsets y*pitch+x) and n_valid [1];
 * scored [3], caller-zeroed, added to by the tile-culled scorers over all
 * rounds: [0] (64-point tile, hypothesis) pairs decided by the tile's
 * bounding box, [1] residuals evaluated point by point (64 per undecided
 * pair), [2] those of [1] evaluated on the matrix cores. */
typedef struct {
    int32_t* counts;
    float* hyps;
    int32_t* triples;
    int32_t* round_info;
    uint8_t* masks;
    int32_t* valid_list;
    int32_t* n_valid;
    unsigned long long* scored;
} pp_ransac_debug;

/* ---------------------------------------------------------------- context */
/* Create a context on HIP device `device`.  PP_E_NODEVICE without a GPU. */
pp_status pp_ctx_create(int32_t device, pp_ctx** out);
/* Wait for the context's outstanding work, free its scratch, destroy it. */
pp_status pp_ctx_destroy(pp_ctx* ctx);
const char* pp_status_string(pp_status s);
/* Text of the last failure on ctx (when ctx is NULL: of the calling thread's last
 * failing pp_ctx_create or pp_ransac_planes_noalloc). */
const char* pp_last_error(const pp_ctx* ctx);

/* ---------------------------------------------------------------- stages */
/* Step 1 (Eq. 1, Alg. 1): N explicit Perona-Malik iterations on the uint16
 * depth image depth_dev [height][pitch]; out_mm_dev [height][pitch] float mm.
 * Per-edge flux lambda * g(I_q - I_p) (I_q - I_p) over the 4 neighbours,
 * zero flux across the border and into holes; holes stay 0. */
pp_status pp_diffuse(pp_ctx* ctx, const uint16_t* depth_dev, float* out_mm_dev, pp_frame_desc desc,
                     const pp_diffuse_params* params, void* hip_stream);

/* Steps 2-3 (Alg. 2 back-projection; Eq. 2, Alg. 1 normals): from float depth
 * in mm, points_dev [3][h][pitch] = z((u-cx)/fx, (v-cy)/fy, 1) metres (0 at
 * holes), normals_dev [3][h][pitch] = -(Sx P x Sy P)/|.| with 3x3 Sobel sums
 * of the point image, valid_dev [h][pitch]: bit0 depth > 0, bit1 normal
 * valid (all 9 neighbours inside and valid, non-zero cross product). */
pp_status pp_normals(pp_ctx* ctx, const float* depth_mm_dev, pp_frame_desc desc, pp_intrinsics K,
                     float* points_dev, float* normals_dev, uint8_t* valid_dev, void* hip_stream);

/* Step 4 (Alg. 2, Eq. 3): sequential whole-frame RANSAC over the depth-valid
 * points (valid bit0).  Round r: hypotheses, inlier counts, j* = most
 * inliers (ties: lowest index), least-squares refit on j*'s inliers (FP64
 * moments + 3x3 eigen-solve), F = refit plane's inliers; if |F| >=
 * min_inliers, planes_dev[r] is written and labels_dev[F] = r, else the
 * frame stops.  Also stops with no valid hypothesis, after max_planes, or
 * with fewer than 3 points left.  labels_dev [h][pitch] int8 (-1 none);
 * n_planes_dev [1].
 *
 * With region_dev_or_null [h][pitch] int16 set, region mode (Alg. 2 as
 * printed; the labels stand for the polygon contours it takes): region g,
 * 0 <= g < max_planes, is the row-major list of depth-valid pixels labelled g
 * (other labels belong to no region).  Per region, hyps_per_plane hypotheses
 * draw three distinct list positions (Philox4x64-10, key (seed, frame_id),
 * counter (j, g, b, 1), position floor(w n_g / 2^64)); each scores
 * error_j = sum of |n.p + d| over all the region's points and its inliers
 * |n.p + d| < thresh_m; the first hypothesis with the smallest error is kept
 * and stored iff inliers / n_g > 0.9 (10 inliers > 9 n_g).  planes_dev [g]
 * (max_planes records) holds region g's kept model (the FP32 hypothesis
 * plane, its inlier count, and the centroid of its inliers when stored);
 * hyp_index is j when stored, -1 otherwise.  labels_dev = g on the inliers
 * of stored regions, -1 elsewhere; n_planes_dev = regions stored.
 * min_inliers and recheck_band_m are unused there; precision must be
 * PP_SCORE_FP32 (else PP_E_UNSUPPORTED).  Scratch grows on first use per
 * shape (may allocate and synchronise the device then). */
pp_status pp_ransac_planes(pp_ctx* ctx, const float* points_dev, const uint8_t* valid_dev,
                           const int16_t* region_dev_or_null, pp_frame_desc desc, const pp_ransac_params* params,
                           pp_plane* planes_dev, int32_t* n_planes_dev, int8_t* labels_dev, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * sequential whole-frame mode of pp_ransac_planes (same kernels, same
 * results for the same arguments) with no context and no allocation.  Its
 * scratch is a device array of PP_NOALLOC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on until the process ends; a frame needing more
 * (about 45.6 bytes per pixel plus 48 per hypothesis: 1280x1024 at 8192
 * hypotheses fits, 1920x1080 does not) returns PP_E_INVAL before any work.
 * Runs on the calling thread's current HIP device with the default tuning,
 * asynchronously on hip_stream; arguments as pp_ransac_planes (no region
 * image).  All calls on one GPU share that array and each call leaves its
 * contents behind: calls whose work may overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.  Errors: PP_E_INVAL
 * for bad arguments, PP_E_HIP for a failed launch (nothing to poison);
 * pp_last_error(NULL) on the calling thread gives the text.  The first call
 * on a device looks the array up (hipGetSymbolAddress). */
#define PP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pp_status pp_ransac_planes_noalloc(const float* points_dev, const uint8_t* valid_dev, pp_frame_desc desc,
                                   const pp_ransac_params* params, pp_plane* planes_dev, int32_t* n_planes_dev,
                                   int8_t* labels_dev, void* hip_stream);

/* Segmentation of the normal image (Sec. III-D: Canny edges on the normal
 * image; the regions between them are the planes region-mode RANSAC fits).
 * From normals_dev [3][h][pitch] and valid_dev bit1 (normal valid):
 *  - the 3x3 Sobel sums of each normal channel give the structure tensor
 *    Exx, Eyy, Exy; m2 = Exx + Eyy is the squared gradient magnitude and the
 *    sector of (Exx - Eyy, 2 Exy) the gradient direction (4 sectors); a pixel
 *    whose 3x3 window holds an invalid normal (or that lies on the border) is
 *    a barrier: no gradient, no edge, no region;
 *  - non-maximum suppression keeps m2 > m2(behind) and m2 >= m2(ahead) along
 *    the sector; weak m2 > low^2, strong m2 > high^2; hysteresis keeps weak
 *    pixels 8-connected to a strong one (edges_dev_or_null [h][pitch] u8);
 *  - regions are the 4-connected components of valid, non-barrier pixels
 *    with no edge pixel in their 3x3 window; those of at least min_area
 *    pixels are numbered 0, 1, ... by size (ties: smallest row-major pixel
 *    index first), at most max_regions; region_dev [h][pitch] int16 (-1
 *    elsewhere), n_regions_dev [1].
 * Every floating-point decision is taken in FP32, so the result is exact
 * and deterministic.  0 <= low <= high; 1 <= max_regions <= 32767;
 * min_area >= 1 with width*height <= 4096 min_area.  Scratch grows on first
 * use per shape (may allocate and synchronise the device then). */
typedef struct { float low; float high; int32_t min_area; int32_t max_regions; } pp_segment_params;
pp_status pp_segment(pp_ctx* ctx, const float* normals_dev, const uint8_t* valid_dev, pp_frame_desc desc,
                     const pp_segment_params* params, int16_t* region_dev, int32_t* n_regions_dev,
                     uint8_t* edges_dev_or_null, void* hip_stream);

/* The contours of regions 0..n_regions-1 of a host label image region_host
 * [height][pitch] int16 (pp_segment's output, copied to the host),
 * simplified into polygons (Sec. III-D).  Contour: the outer boundary,
 * traced with the Moore neighbourhood clockwise on screen from the region's
 * first pixel in row-major order (entered from the west) until the trace is
 * back on the start and its next move would repeat the first move.  Simplification: Douglas-Peucker on the
 * closed contour split at the point farthest from the start; a point stays
 * iff its distance to the chord exceeds eps_px.  Output: xy_host
 * [max_vertices][2] int32 (x = column, y = row), offsets_host [n_regions+1]
 * (region g's vertices are offsets[g] .. offsets[g+1]-1; none for an empty
 * region).  Host memory only, no device work.  PP_E_NOMEM when max_vertices
 * is too small: offsets_host[n_regions] then holds the number needed and
 * nothing past max_vertices is written. */
pp_status pp_region_polygons(const int16_t* region_host, pp_frame_desc desc, int32_t n_regions, double eps_px,
                             int32_t* xy_host, int32_t max_vertices, int32_t* offsets_host);

/* ---------------------------------------------------------------- map */
/* Polygon map with vertical drift compensation (Sec. III-E, Eqs. 4-10), host
 * code in float64.  The map keeps near-horizontal polygons (normal within
 * max_tilt_deg of world +Z; the others are skipped).  pp_map_integrate takes
 * one frame: the camera pose from odometry (R world<-camera row-major, C the
 * camera centre; its height may drift) and the frame's polygons in the camera
 * frame (plane n.p + d = 0, centroid, support, and the pixel polygon of
 * pp_region_polygons, lifted onto the plane through K).  A polygon's raw
 * height is its centroid's world z.  It matches the map polygon whose
 * footprint (convex hull in world x, y) overlaps its own with positive area
 * and whose height is within drift_tolerance_m (Eq. 5; the paper's 5 cm) of
 * the raw height minus the drift estimate; the smallest difference wins,
 * ties to the older map polygon.  The measurement z_k is the mean of raw
 * minus map height over the matches; the drift filter predicts (Eqs. 6-7:
 * P += sigma_p) and, with a measurement, updates (Eqs. 8-10).  The polygons,
 * corrected by the updated estimate, merge into their match (hull of both,
 * support-weighted height, supports add) or are appended, in input order.
 * match_of_out [n] (may be NULL): map index, -1 appended, -2 skipped. */
typedef struct pp_map pp_map;
typedef struct { double drift_tolerance_m; double sigma_p; double sigma_m; double max_tilt_deg; } pp_map_params;
typedef struct {
    double n[3];
    double d;
    double centroid[3];
    int32_t support;
    int32_t n_vertices;
    const int32_t* xy_px; /* [n_vertices][2] (x = column, y = row) */
} pp_map_observation;
typedef struct {
    int32_t matched, added, skipped, pad;
    double measurement; /* z_k, NaN without a match */
    double drift;       /* x_k */
    double variance;    /* P_k */
} pp_map_frame_result;
typedef struct { double height; int64_t support; int32_t n_vertices; int32_t pad; } pp_map_polygon_info;
/* 0 < drift_tolerance_m, 0 <= sigma_p, 0 < sigma_m, 0 <= max_tilt_deg < 90. */
pp_status pp_map_create(const pp_map_params* params, pp_map** out);
pp_status pp_map_destroy(pp_map* map);
pp_status pp_map_integrate(pp_map* map, pp_intrinsics K, const double* R_world_cam, const double* C_world,
                           const pp_map_observation* polygons, int32_t n, int32_t* match_of_out,
                           pp_map_frame_result* out);
pp_status pp_map_size(const pp_map* map, int32_t* n);
/* Map polygon i: height, support, and its footprint's vertices (counter-
 * clockwise, world x, y) into xy_out [max_vertices][2]; PP_E_NOMEM (with
 * info->n_vertices set) when max_vertices is too small. */
pp_status pp_map_polygon(const pp_map* map, int32_t i, pp_map_polygon_info* info, double* xy_out,
                         int32_t max_vertices);

/* pp_ransac_planes that also fills the introspection buffers of *dbg. */
pp_status pp_ransac_planes_dbg(pp_ctx* ctx, const float* points_dev, const uint8_t* valid_dev,
                               pp_frame_desc desc, const pp_ransac_params* params, pp_plane* planes_dev,
                               int32_t* n_planes_dev, int8_t* labels_dev, const pp_ransac_debug* dbg,
                               void* hip_stream);

/* Region-mode introspection (device buffers; any may be NULL), R = max_planes,
 * Hy = hyps_per_plane: npts [R] points per region; triples [R][Hy][3] list
 * positions (-1 when fewer than three were drawn); hyps [R][Hy][4] FP32
 * planes (d = NaN without a plane); errors [R][Hy] FP64 sums of |r|
 * (+inf without a plane); counts [R][Hy] inliers; jstar [R] kept hypothesis
 * (-1 none). */
typedef struct {
    int32_t* npts;
    int32_t* triples;
    float* hyps;
    double* errors;
    int32_t* counts;
    int32_t* jstar;
} pp_region_debug;

/* Region-mode pp_ransac_planes (region_dev must not be NULL) that also fills *dbg. */
pp_status pp_ransac_regions_dbg(pp_ctx* ctx, const float* points_dev, const uint8_t* valid_dev,
                                const int16_t* region_dev, pp_frame_desc desc, const pp_ransac_params* params,
                                pp_plane* planes_dev, int32_t* n_planes_dev, int8_t* labels_dev,
                                const pp_region_debug* dbg, void* hip_stream);

/* Score caller-given triples of pixel offsets (y*pitch+x) against every
 * depth-valid point: planes_dev [n][4] receives each triple's FP32 plane
 * (d = NaN if degenerate), counts_dev [n] its inlier count (Eq. 3, strict <). */
pp_status pp_debug_score_triples(pp_ctx* ctx, const float* points_dev, const uint8_t* valid_dev,
                                 pp_frame_desc desc, const int32_t* triples_dev, int32_t n, float thresh_m,
                                 int32_t precision, float recheck_band_m, float* planes_dev,
                                 int32_t* counts_dev, void* hip_stream);

/* ---------------------------------------------------------------- whole frames */
/* One frame through all four steps.  All pointers are caller device buffers:
 * depth [h][pitch] uint16 in; depth_mm, points, normals, valid, labels,
 * planes [max_planes], n_planes [1] out. */
typedef struct {
    const uint16_t* depth;
    pp_frame_desc desc;
    pp_intrinsics K;
    pp_diffuse_params diffuse;
    pp_ransac_params ransac;
    float* depth_mm;
    float* points;
    float* normals;
    uint8_t* valid;
    pp_plane* planes;
    int32_t* n_planes;
    int8_t* labels;
} pp_frame_job;

/* Host-only check of a job's descriptor, parameters and pointers (non-NULL);
 * makes no HIP call.  PP_OK or PP_E_INVAL. */
pp_status pp_validate_job(const pp_frame_job* job);

/* A ragged batch of frames (any mix of sizes and parameters, one scoring
 * precision per batch) run together:
 * each stage is one launch over all frames, and the whole sequence is
 * captured once per batch layout into a HIP graph and replayed.  Results are
 * bitwise identical to running each frame alone.  jobs is a host array. */
pp_status pp_batch_run(pp_ctx* ctx, int32_t n_frames, const pp_frame_job* jobs, void* hip_stream);

/* Same, without graph capture (plain stream launches). */
pp_status pp_batch_run_eager(pp_ctx* ctx, int32_t n_frames, const pp_frame_job* jobs, void* hip_stream);

/* ---------------------------------------------------------------- tuning */
/* Launch-shape knobs the autotuner searches (0 = library default).
 * diffuse_tile: the diffusion kernel's tile shape (1-4: LDS tiles of 64x16,
 * 128x16, 64x32 and 128x32 pixels; 5, 6: register-resident columns, one
 * wave per 64 - 2T columns and 8 or 16 rows), diffuse_t: iterations fused
 * per pass (temporal blocking depth), score_hb: the scorer's hypotheses per
 * block (1: 8, 2: 16, 3: 32, every point on the vector ALUs, FP32 form only;
 * 4: 64, 5: 128, 6: 256 with tile culling: each 64-point tile's bounding box
 * first decides for every hypothesis whether all, none or only some of its
 * points can be inliers; the matrix-core forms always cull, at 64 when 1-3
 * is set), score_chunk: points per scoring work item.  Every choice gives
 * identical results. */
typedef struct {
    int32_t diffuse_tile;
    int32_t diffuse_t;
    int32_t score_hb;
    int32_t score_chunk;
} pp_tuning;
/* Set (or, with NULL, reset) the context's tuning; invalid knobs: PP_E_INVAL. */
pp_status pp_set_tuning(pp_ctx* ctx, const pp_tuning* tuning);
pp_status pp_get_tuning(const pp_ctx* ctx, pp_tuning* out);
/* Number of choices per knob (for the autotuner's search space). */
pp_status pp_tuning_space(int32_t* n_tiles, int32_t* max_t, int32_t* n_hb, int32_t* n_chunk);

/* ---------------------------------------------------------------- serving */
/* A server runs frames from several camera streams as they arrive.  A
 * scheduler thread admits queued frames in arrival order whenever their
 * device block (inputs, outputs and scratch) fits the HBM budget, groups the
 * admitted frames into ragged batches of up to max_batch, and launches each
 * batch (all four steps, pp_batch_run) on one of `lanes` HIP streams, so
 * frames arriving while others run are admitted as memory frees up and
 * overlap with them on the device.  A frame's results do not depend on what
 * it was batched with.  pp_submit and pp_poll are thread-safe. */
typedef struct pp_server pp_server;

typedef struct {
    int32_t device;
    uint64_t hbm_budget_bytes;  /* arena for frames in flight, allocated once at create */
    int32_t max_batch;          /* frames per launch, 1..1024 */
    int32_t lanes;              /* batches in flight at once, 1..4 */
    int32_t staging_frames;     /* pinned host slots per stream (queued + unpolled frames), 1..1024 */
    int32_t use_graphs;         /* 1: replay cached HIP graphs per batch layout; 0: eager launches */
    int32_t dry_run_us;         /* > 0: no GPU is touched; each batch "completes" after this many us
                                   with no planes -- exercises admission and scheduling only */
    int32_t dry_run_fail_batch; /* dry run only: the n-th launched batch (1-based) ends as a failed
                                   HIP batch would, poisoning the server; 0: never */
} pp_server_cfg;

/* Caller-owned host buffers filled by pp_poll. */
typedef struct {
    pp_plane* planes;     /* [max_planes] of the frame's stream (NULL: skip) */
    int32_t* n_planes;    /* [1] (NULL: skip) */
    int8_t* labels;       /* [height*width] (NULL: skip) */
    int32_t stream_id;
    uint64_t frame_id;
    double latency_us;    /* pp_submit -> results on the host */
} pp_result;

typedef struct {
    uint64_t submitted, completed, rejected, cancelled, launches;
    double mean_batch;            /* frames per launch */
    double p50_us, p99_us, max_us;/* latency of completed frames (last 65536) */
    uint64_t hbm_in_use, hbm_peak;/* arena bytes */
    int32_t queued, in_flight;
} pp_server_stats;

/* PP_E_INVAL for bad cfg, PP_E_NODEVICE without a GPU (unless dry_run_us > 0). */
pp_status pp_server_create(const pp_server_cfg* cfg, pp_server** out);
/* Stops the scheduler, waits for batches on the device, frees everything. */
pp_status pp_server_destroy(pp_server* s);
/* Text of the failure that poisoned the server ("" if none); the pointer stays
 * valid until the calling thread's next call. */
const char* pp_server_last_error(const pp_server* s);
/* Register camera stream stream_id (unique for the server's lifetime): frame
 * size (pitch_px == width), intrinsics and parameters.  PP_E_BUDGET if one
 * frame of it can never fit the budget. */
pp_status pp_stream_open(pp_server* s, int32_t stream_id, pp_frame_desc desc, pp_intrinsics K,
                         const pp_diffuse_params* dp, const pp_ransac_params* rp);
/* Queued frames of the stream are cancelled (their polls return PP_E_CLOSED);
 * launched frames complete and stay pollable. */
pp_status pp_stream_close(pp_server* s, int32_t stream_id);
/* Copy a host uint16 [height][width] frame into pinned staging and queue it;
 * never blocks.  frame_id keys the frame's hypotheses.  *ticket identifies
 * the result.  PP_E_AGAIN when the stream's staging is full; PP_E_CLOSED if
 * the stream is (or was meanwhile) closed; PP_E_HIP once a failure has
 * poisoned the server (also when it happens while the frame is copied: the
 * frame is then not queued). */
pp_status pp_submit(pp_server* s, int32_t stream_id, const uint16_t* depth_host, uint64_t frame_id,
                    uint64_t* ticket);
/* Wait up to timeout_us (0: don't wait) for the ticket: PP_OK with the results
 * copied into *out (the ticket is then released), PP_PENDING if not ready,
 * PP_E_CLOSED if cancelled, PP_E_HIP if its batch failed. */
pp_status pp_poll(pp_server* s, uint64_t ticket, pp_result* out, int32_t timeout_us);
pp_status pp_server_stats_get(pp_server* s, pp_server_stats* out);
/* Clear a server (poisoned or not) for new work: waits for the batches on
 * the device, fails every frame not yet completed (its poll returns
 * PP_E_HIP if the server was poisoned, PP_E_CLOSED otherwise), frees their
 * memory, gives every lane a fresh context, and accepts frames again.  Open
 * streams stay open; completed results stay pollable.  PP_E_HIP (still
 * poisoned) if the device cannot take new contexts. */
pp_status pp_server_reset(pp_server* s);

/* ---------------------------------------------------------------- timing */
/* Stage timing: while enabled, every launch of the inlier-scoring kernel
 * (one per RANSAC round) made by pp_ransac_planes or pp_batch_run_eager is
 * bracketed by HIP events recorded on the launching stream (graph replays of
 * pp_batch_run are not instrumented).  pp_stage_time returns the summed
 * elapsed ms of those launches in the most recent instrumented run on ctx and
 * their number; the caller must have synchronised the stream first. */
pp_status pp_set_stage_timing(pp_ctx* ctx, int32_t enable);
pp_status pp_stage_time(pp_ctx* ctx, float* total_ms, int32_t* launches);
/* For the most recent instrumented pp_batch_run_eager: ms of [0] diffusion,
 * [1] back-projection + normals + valid list, [2] inlier scoring (all
 * rounds), [3] the rest of RANSAC (hypotheses, refit, labelling). */
pp_status pp_stage_breakdown(pp_ctx* ctx, float out_ms[4]);

#ifdef __cplusplus
}
#endif
#endif /* PP_H */
