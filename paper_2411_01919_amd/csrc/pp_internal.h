// Internal declarations shared by the kernels (pp_kernels.hip) and the C ABI
// (pp_api.hip) of libpp.so.  Not installed; the public interface is pp.h.
#pragma once

#include <cstddef>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pp.h"

namespace ppk {

constexpr int kMaxRounds = 127;   // labels are int8
constexpr int kMaxHyps = 8192;
constexpr int kBlock = 256;       // threads per workgroup (4 wave64s)
constexpr int kValidChunk = 1024; // pixels per valid-list chunk
constexpr int kRefitChunk = 2048; // points per refit / apply chunk
constexpr int kScanBlock = 8;     // the scoring list walks the image in 8x8-pixel blocks

// Per-frame RANSAC state in device memory.  Fields indexed by the round r are
// written only by an earlier kernel than the ones that read them, so no
// kernel reads a field another block of the same launch may be writing.
// One round's flags, read together by a single 32-byte scalar load.
struct RoundRec {
    int32_t active;  // round r runs iff active
    int32_t M;       // |R_r|: unassigned points entering round r
    int32_t stop;    // round r found no valid hypothesis
    int32_t jstar;
    int32_t Mlen;    // length of round r's point list: R_r in order, each chunk's run padded with NaN points
                     // to a multiple of 64 (every 64-point tile lies inside one chunk's run)
    int32_t pad[3];
};

struct RoundState {
    int32_t M0;                        // |L|: depth-valid pixels
    uint32_t p1max_bits;               // max |x|+|y|+|z| over the frame's points (float bits)
    int32_t s_count;
    int32_t pad[5];
    RoundRec round[kMaxRounds + 1];
    double plane[4];                   // refit plane of the current round
    double centroid[3];
};
static_assert(offsetof(RoundState, M0) == 0 && offsetof(RoundState, round) % 32 == 0, "RoundState layout");

// Everything a kernel needs about one frame.  Kernels read a table of these
// from device memory and take the frame index from blockIdx.z.
struct FrameDev {
    // caller buffers
    const uint16_t* depth;   // [H][pitch]
    float* dmm;              // [H][pitch] diffused depth, mm
    float* pts;              // [3][H][pitch] metres
    float* nrm;              // [3][H][pitch]
    uint8_t* valid;          // [H][pitch]
    int8_t* labels;          // [H][pitch]
    pp_plane* planes;        // [max_planes]
    int32_t* n_planes;       // [1]
    // geometry
    int32_t W, H, pitch, pad0;
    float fx, fy, cx, cy;
    float ifx, ify;          // 1/fx, 1/fy (correctly rounded, set on the host)
    // diffusion
    int32_t iters;
    float lambda;
    float g_scale;           // exp form: log2(e)/kappa^2 ; rational: 1/kappa^2
    int32_t edge_stop;
    int32_t scheme;  // PP_DIFFUSE_*
    // RANSAC
    int32_t max_planes, hyps, min_inliers, precision;
    float thresh, band;
    uint64_t seed, frame_id;
    // library scratch
    float* delta[2];         // [H][W] diffusion ping-pong (delta = I - I0)
    int32_t* L;              // [W*H] valid list (pixel offsets y*pitch+x)
    float4* list[2];         // [scan positions] remaining points (x, y, z, valid-list position bits), NaN padding
    uint8_t* taken;          // [W*H] 1 iff the point at valid-list position k is assigned
    float4* hyp;             // [hyps] (n, d); d = NaN when invalid
    float4* hyp_p0;          // [hyps] the first point of each hypothesis' triple (the refit's moment origin)
    int32_t* triples;        // [hyps][3]
    int32_t* counts;         // [hyps]
    double* partials;        // [refit chunks][10]
    int32_t* chunk_cnt;      // [max(valid chunks, refit chunks)]
    float4* tbox;            // [list tiles][2] per 64-point tile of the current list: centre (w: count of
                             // its points that are not padding) and half extents of their bounding box
    int32_t* chunk_run;      // [refit chunks] padded length of each chunk's run of survivors
    RoundState* st;
    // introspection (may be null)
    pp_ransac_debug dbg;
};

struct Tuning {
    int diffuse_tile;  // LDS tiles 64x16, 128x16, 64x32, 128x32; register-resident waves of TY = 8, 16 rows
    int diffuse_t;     // iterations per pass
    int score_hb;      // index into {8, 16, 32, then 64, 128, 256 with tile culling (1, 2, 4 per lane)}
    int score_chunk;   // index into {1024, 2048, 4096, 8192}
};

constexpr int kNumTiles = 6;
constexpr int kMaxT = 10;
constexpr int kNumHB = 6;
constexpr int kNumChunk = 4;
int hb_value(int idx);
int chunk_value(int idx);
bool t_supported(int t);

// Launchers (all asynchronous on `s`).  `tab` is a device array of nf frames;
// the *max* arguments bound the per-frame sizes and size the grids.
hipError_t launch_diffuse(const FrameDev* tab, int nf, int maxW, int maxH, int iters_max, int scheme,
                          const Tuning& tu, hipStream_t s);
// count: the normals pass also writes the valid-list chunk counts, and the
// following launch_valid_list is then called with counted = true
hipError_t launch_normals(const FrameDev* tab, int nf, int max_px, bool count, hipStream_t s);
hipError_t launch_valid_list(const FrameDev* tab, int nf, int max_px, int maxW, int maxH, bool counted, hipStream_t s);
hipError_t launch_round(const FrameDev* tab, int nf, int r, int max_px, int max_hyps, int precision,
                        const Tuning& tu, hipStream_t s, hipEvent_t score_start = nullptr,
                        hipEvent_t score_end = nullptr);
// Positions of the 8x8-block scan of a W x H frame (whole blocks): the length
// of its round-0 point list, which no later round's list exceeds, and at
// least W H.  Frame scratch is sized by it.
inline size_t scan_pixels(int W, int H) { return (size_t)((W + 7) / 8) * (size_t)((H + 7) / 8) * 64; }
hipError_t launch_hyp_from_triples(const FrameDev* tab, const int32_t* triples, int n, hipStream_t s);
hipError_t launch_score_only(const FrameDev* tab, int max_px, int n, int precision, const Tuning& tu,
                             hipStream_t s);

// Region mode (Alg. 2 as printed): one frame per call, plain calls only.
constexpr int kRegionPxChunk = 4096;  // pixels per list-building block
constexpr int kRegionChunk = 512;     // region points per scoring block

struct RegionDev {
    const float* pts;        // [3][H][pitch]
    const uint8_t* valid;    // [H][pitch] bit0: depth
    const int16_t* region;   // [H][pitch] region labels
    int32_t W, H, pitch;
    int32_t R, hyps, nb;     // regions, hypotheses per region, list-building blocks
    float thresh;
    int32_t pad;
    uint64_t seed, frame_id;
    // scratch (region_bind_scratch)
    int32_t* bcnt;           // [nb][R] points per (block, region), then list positions
    int32_t* off;            // [R+1] first list position of each region
    int32_t* choff;          // [R+1] first scoring chunk of each region
    int32_t* npts;           // [R]
    int32_t* list;           // [W*H] pixel offsets grouped by region, row-major within
    float4* hyp;             // [R][hyps] FP32 planes (n, d); d = NaN without a plane
    int32_t* triples;        // [R][hyps][3] list positions (-1: fewer than 3 drawn)
    double* errp;            // [chunks][hyps] per-chunk sums of |r|
    int32_t* counts;         // [R][hyps]
    double* errors;          // [R][hyps]
    int32_t* jstar;          // [R]
    double* cpart;           // [chunks][3] partial sums of the inliers' coordinates
    // caller outputs
    pp_plane* planes;        // [R]
    int32_t* n_planes;
    int8_t* labels;          // [H][pitch]
};

int region_blocks(int W, int H);
int region_max_chunks(int W, int H, int R);
size_t region_bind_scratch(RegionDev& r, void* scratch);  // returns the bytes used
size_t region_scratch_bytes(int W, int H, int R, int hyps);
hipError_t launch_regions(const RegionDev& r, hipStream_t s);

// Segmentation of the normal image (one frame per call).
constexpr int kSegMaxCand = 4096;  // components of at least min_area pixels (W*H / min_area bounds them)

struct SegDev {
    const float* nrm;        // [3][H][pitch] normals
    const uint8_t* valid;    // [H][pitch] bit1: normal valid
    int32_t W, H, pitch, min_area, max_regions;
    float low, high;         // thresholds on the gradient magnitude
    int16_t* region;         // [H][pitch] out: -1 or rank
    int32_t* n_regions;      // [1] out
    uint8_t* edges;          // [H][pitch] out, may be null
    // scratch (seg_bind_scratch), [H][W] unless noted
    float* m2;
    int32_t* root;           // aliases m2 (dead after suppression)
    uint8_t* meta;           // sector | barrier | weak | strong | edge bits
    uint8_t* strong;         // by union-find root: the edge component holds a strong pixel
    int32_t* parent;         // union-find of edge pixels
    int32_t* parent2;        // union-find of region pixels
    int32_t* cnt;            // component size by root
    int32_t* rank;           // region label by root
    unsigned long long* cand;  // [kSegMaxCand]
    int32_t* ncand;          // [1]
};

size_t seg_bind_scratch(SegDev& s, void* scratch);  // returns the bytes used
size_t seg_scratch_bytes(int W, int H);
hipError_t launch_segment(const SegDev& s, hipStream_t st);

// Library scratch one frame needs (the server carves it from its arena), and
// a batch run whose frame slots use caller-provided scratch (scratch[i] for
// jobs[i], each frame_scratch_bytes() long).
size_t frame_scratch_bytes(int width, int height, int hyps);
pp_status batch_run_external(pp_ctx* c, int n, const pp_frame_job* jobs, void* const* scratch, hipStream_t s,
                             bool graph);
const char* ctx_error(const pp_ctx* c);

}  // namespace ppk
