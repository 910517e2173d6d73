// C ABI of libpp.so: contexts, argument checks, scratch management and the
// launch sequences of the plain (per-stage), per-frame and batched paths.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pp_internal.h"

using ppk::FrameDev;
using ppk::RoundState;

namespace {

thread_local std::string g_create_error;

// Library scratch of one frame slot, carved out of a single allocation.
struct Slot {
    void* base = nullptr;
    size_t bytes = 0;
    size_t px_cap = 0;
    int hyp_cap = 0;
    bool external = false;  // memory owned by the caller (the server's arena)
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after the latest launch of exec
    uint64_t last_use = 0;
};

// Captured graphs kept per context (least recently used ones are destroyed
// beyond this; a server sees one layout per batch size and frame mix).
constexpr size_t kMaxGraphs = 64;

}  // namespace

// register-resident diffusion (16 rows a wave), 4 iterations a pass, the culled scorer, 2048 points a scoring block
constexpr ppk::Tuning kDefaultTuning{5, 4, 3, 1};

struct pp_ctx {
    int device = 0;
    bool poisoned = false;
    std::string last_error;
    ppk::Tuning tuning = kDefaultTuning;
    std::vector<Slot> slots;
    // device frame tables: [0] single-frame calls, [1] batches
    FrameDev* plain_tab = nullptr;
    FrameDev* batch_tab = nullptr;
    int batch_tab_cap = 0;
    // pinned staging for batch tables (ring, one event per entry)
    static constexpr int kRing = 8;
    FrameDev* staging[kRing] = {nullptr};
    int staging_cap[kRing] = {0};
    hipEvent_t staging_ev[kRing] = {nullptr};
    bool staging_used[kRing] = {false};
    int ring_pos = 0;
    hipStream_t capture_stream = nullptr;
    // a batch's frames run as up to kMaxChains independent kernel chains: chain 0 on
    // the launching stream, the others on these, forked and joined by events
    static constexpr int kMaxChains = 4;
    bool chains = true;  // false: every batch runs as one chain (the serving runtime's contexts)
    hipStream_t chain_stream[kMaxChains] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kMaxChains] = {};
    std::map<std::string, GraphEntry> graphs;
    uint64_t graph_clock = 0;
    // the stream of the latest enqueue and an event after it: a call on
    // another stream first waits for it (the frame tables and scratch are shared)
    hipStream_t last_stream = nullptr;
    hipEvent_t last_ev = nullptr;
    bool last_valid = false;
    void* debug_scratch = nullptr;
    size_t debug_scratch_bytes = 0;
    void* region_scratch = nullptr;
    size_t region_scratch_bytes = 0;
    void* seg_scratch = nullptr;
    size_t seg_scratch_bytes = 0;
    // stage timing: events around each round's scoring launch
    bool timing = false;
    hipEvent_t score_ev[ppk::kMaxRounds][2] = {};
    hipEvent_t stage_ev[4] = {};  // batch start, after diffusion, after normals + valid list, end
    bool stages_valid = false;
    int timed_rounds = 0;
};

namespace {

pp_status fail(pp_ctx* c, pp_status s, const std::string& msg) {
    if (c) {
        c->last_error = msg;
        if (s == PP_E_HIP) c->poisoned = true;
    } else {
        g_create_error = msg;
    }
    return s;
}

pp_status hip_fail(pp_ctx* c, hipError_t e, const char* where) {
    return fail(c, PP_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, call)                                        \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
    } while (0)

// Destroy one captured graph once its latest launch has finished.
void destroy_graph(GraphEntry& g) {
    if (g.done) {
        (void)hipEventSynchronize(g.done);
        (void)hipEventDestroy(g.done);
    }
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    g.done = nullptr;
}

void drop_graphs(pp_ctx* c) {
    for (auto& kv : c->graphs) destroy_graph(kv.second);
    c->graphs.clear();
}

// Work enqueued on one context's shared tables and scratch stays in order
// across streams: a call on a stream other than the previous call's waits
// for the previous call's work first.
// A stream under the caller's graph capture is left alone (an event
// recorded there is not a recorded event afterwards): the capturing caller
// orders its own graph.
bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

pp_status order_streams(pp_ctx* c, hipStream_t st) {
    if (c->last_valid && st != c->last_stream && !capturing(st)) HIPCHK(c, hipStreamWaitEvent(st, c->last_ev, 0));
    return PP_OK;
}

pp_status mark_stream(pp_ctx* c, hipStream_t st) {
    if (capturing(st)) {
        c->last_valid = false;
        return PP_OK;
    }
    HIPCHK(c, hipEventRecord(c->last_ev, st));
    c->last_stream = st;
    c->last_valid = true;
    return PP_OK;
}

bool desc_ok(const pp_frame_desc& d) {
    return d.width >= 3 && d.height >= 3 && d.width <= 16384 && d.height <= 16384 && d.pitch_px >= d.width &&
           (int64_t)d.width * d.height <= (int64_t(1) << 27) && (int64_t)d.pitch_px * d.height <= (int64_t(1) << 30);
}

bool diffuse_params_ok(const pp_diffuse_params* p) {
    if (!p || p->scheme < PP_DIFFUSE_EDGE4 || p->scheme > PP_DIFFUSE_EDGE8) return false;
    const float lam_max = p->scheme == PP_DIFFUSE_EDGE8 ? 1.0f / 6.0f : 0.25f;
    return p->iters >= 0 && p->iters <= 1000 && p->lambda > 0.f && p->lambda <= lam_max && p->kappa_mm > 0.f &&
           isfinite(p->lambda) && (p->edge_stop == PP_EDGE_EXP || p->edge_stop == PP_EDGE_RATIONAL);
}

bool ransac_params_ok(const pp_ransac_params* p) {
    return p && p->max_planes >= 1 && p->max_planes <= ppk::kMaxRounds && p->hyps_per_plane >= 1 &&
           p->hyps_per_plane <= ppk::kMaxHyps && p->min_inliers >= 1 && p->thresh_m > 0.f && isfinite(p->thresh_m) &&
           p->precision >= PP_SCORE_FP32 && p->precision <= PP_SCORE_FP16 && p->recheck_band_m >= 0.f &&
           isfinite(p->recheck_band_m);
}

bool intrinsics_ok(const pp_intrinsics& K) {
    return K.fx > 0.f && K.fy > 0.f && isfinite(K.fx) && isfinite(K.fy) && isfinite(K.cx) && isfinite(K.cy);
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
    size_t delta, L, list, taken, hyp, hyp_p0, triples, counts, partials, chunk_cnt, tbox, chunk_run, st, total;
};

// px: the slot's pixel capacity, at least the scan positions of every frame it
// holds (ppk::scan_pixels), which is also its point lists' capacity.
Layout slot_layout(size_t px, int hyps) {
    Layout l;
    const size_t nch_refit = (px + ppk::kRefitChunk - 1) / ppk::kRefitChunk;
    const size_t nch_valid = (px + ppk::kValidChunk - 1) / ppk::kValidChunk;
    size_t o = 0;
    l.delta = o; o += align256(2 * px * sizeof(float));
    l.L = o; o += align256(px * sizeof(int32_t));
    l.list = o; o += align256(2 * px * sizeof(float4));
    l.taken = o; o += align256(px);
    l.hyp = o; o += align256((size_t)hyps * sizeof(float4));
    l.hyp_p0 = o; o += align256((size_t)hyps * sizeof(float4));
    l.triples = o; o += align256((size_t)hyps * 3 * sizeof(int32_t));
    l.counts = o; o += align256((size_t)hyps * sizeof(int32_t));
    l.partials = o; o += align256(nch_refit * 10 * sizeof(double));
    l.chunk_cnt = o; o += align256(std::max(nch_refit, nch_valid) * sizeof(int32_t));
    l.tbox = o; o += align256((px + 63) / 64 * 2 * sizeof(float4));
    l.chunk_run = o; o += align256(nch_refit * sizeof(int32_t));
    l.st = o; o += align256(sizeof(RoundState));
    l.total = o;
    return l;
}

// Make slot i big enough for px pixels and hyps hypotheses.  Growing waits
// for the device first: earlier work may still use the old buffers.
pp_status ensure_slot(pp_ctx* c, int i, size_t px, int hyps) {
    if ((int)c->slots.size() <= i) c->slots.resize(i + 1);
    Slot& s = c->slots[i];
    if (s.base && s.px_cap >= px && s.hyp_cap >= hyps) return PP_OK;
    if (s.external) return fail(c, PP_E_INVAL, "external scratch too small for the frame");
    const size_t npx = std::max(px, s.px_cap);
    const int nh = std::max(hyps, s.hyp_cap);
    Layout l = slot_layout(npx, nh);
    if (s.base) {
        HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipFree(s.base));
        s.base = nullptr;
    }
    hipError_t e = hipMalloc(&s.base, l.total);
    if (e != hipSuccess) {
        s.base = nullptr;
        s.px_cap = 0;
        s.hyp_cap = 0;
        (void)hipGetLastError();
        return fail(c, PP_E_NOMEM, "hipMalloc of frame scratch failed");
    }
    s.bytes = l.total;
    s.px_cap = npx;
    s.hyp_cap = nh;
    return PP_OK;
}

// Point a frame's scratch fields into one block laid out by slot_layout(px_cap, hyp_cap).
void bind_layout(char* b, size_t px_cap, int hyp_cap, FrameDev& f) {
    Layout l = slot_layout(px_cap, hyp_cap);
    f.delta[0] = reinterpret_cast<float*>(b + l.delta);
    f.delta[1] = f.delta[0] + px_cap;
    f.L = reinterpret_cast<int32_t*>(b + l.L);
    f.list[0] = reinterpret_cast<float4*>(b + l.list);
    f.list[1] = f.list[0] + px_cap;
    f.taken = reinterpret_cast<uint8_t*>(b + l.taken);
    f.hyp = reinterpret_cast<float4*>(b + l.hyp);
    f.hyp_p0 = reinterpret_cast<float4*>(b + l.hyp_p0);
    f.triples = reinterpret_cast<int32_t*>(b + l.triples);
    f.counts = reinterpret_cast<int32_t*>(b + l.counts);
    f.partials = reinterpret_cast<double*>(b + l.partials);
    f.chunk_cnt = reinterpret_cast<int32_t*>(b + l.chunk_cnt);
    f.tbox = reinterpret_cast<float4*>(b + l.tbox);
    f.chunk_run = reinterpret_cast<int32_t*>(b + l.chunk_run);
    f.st = reinterpret_cast<RoundState*>(b + l.st);
}

void bind_slot(const pp_ctx* c, int i, FrameDev& f) {
    const Slot& s = c->slots[i];
    bind_layout(static_cast<char*>(s.base), s.px_cap, s.hyp_cap, f);
}

void fill_geometry(FrameDev& f, const pp_frame_desc& d) {
    f.W = d.width;
    f.H = d.height;
    f.pitch = d.pitch_px;
}

void fill_diffuse(FrameDev& f, const pp_diffuse_params& p) {
    f.iters = p.iters;
    f.lambda = p.lambda;
    f.edge_stop = p.edge_stop;
    f.scheme = p.scheme;
    const double k2 = (double)p.kappa_mm * (double)p.kappa_mm;
    // exp(-(x/k)^2) = 2^(-x^2 log2(e)/k^2); as k -> inf the scale underflows to 0 and g == 1
    f.g_scale = (float)(p.edge_stop == PP_EDGE_RATIONAL ? 1.0 / k2 : 1.4426950408889634 / k2);
}

void fill_ransac(FrameDev& f, const pp_ransac_params& p) {
    f.max_planes = p.max_planes;
    f.hyps = p.hyps_per_plane;
    f.min_inliers = p.min_inliers;
    f.precision = p.precision;
    f.thresh = p.thresh_m;
    f.band = p.recheck_band_m;
    f.seed = p.seed;
    f.frame_id = p.frame_id;
}

__global__ void k_set_frame(FrameDev* dst, FrameDev v) { *dst = v; }

__global__ void k_force_active(FrameDev* tab) {
    RoundState* st = tab[0].st;
    st->round[0].active = st->M0 > 0 ? 1 : 0;
}

pp_status put_plain(pp_ctx* c, const FrameDev& f, hipStream_t s) {
    pp_status ps = order_streams(c, s);
    if (ps != PP_OK) return ps;
    hipLaunchKernelGGL(k_set_frame, dim3(1), dim3(1), 0, s, c->plain_tab, f);
    HIPCHK(c, hipGetLastError());
    return PP_OK;
}

pp_status check_ctx(pp_ctx* c) {
    if (!c) return PP_E_INVAL;
    if (c->poisoned) return PP_E_HIP;
    return PP_OK;
}

pp_status set_device(pp_ctx* c) {
    HIPCHK(c, hipSetDevice(c->device));
    return PP_OK;
}

}  // namespace

// =====================================================================
extern "C" {

const char* pp_status_string(pp_status s) {
    switch (s) {
        case PP_OK: return "ok";
        case PP_PENDING: return "pending";
        case PP_E_INVAL: return "invalid argument";
        case PP_E_NOMEM: return "out of device memory";
        case PP_E_BUDGET: return "exceeds the HBM budget";
        case PP_E_HIP: return "HIP runtime error";
        case PP_E_NODEVICE: return "no GPU device";
        case PP_E_CLOSED: return "closed";
        case PP_E_UNSUPPORTED: return "unsupported";
        case PP_E_TIMEOUT: return "timed out";
        default: return "unknown status";
    }
}

const char* pp_last_error(const pp_ctx* c) { return c ? c->last_error.c_str() : g_create_error.c_str(); }

pp_status pp_ctx_create(int32_t device, pp_ctx** out) {
    if (!out) return PP_E_INVAL;
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(nullptr, PP_E_NODEVICE, "no HIP device available");
    }
    if (device < 0 || device >= n) return fail(nullptr, PP_E_INVAL, "device index out of range");
    pp_ctx* c = new pp_ctx();
    c->device = device;
    e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc(&c->plain_tab, sizeof(FrameDev));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    for (int i = 0; e == hipSuccess && i < pp_ctx::kRing; ++i) e = hipEventCreateWithFlags(&c->staging_ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->last_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        g_create_error = std::string("context set-up failed: ") + hipGetErrorString(e);
        pp_ctx_destroy(c);
        return e == hipErrorOutOfMemory ? PP_E_NOMEM : PP_E_HIP;
    }
    *out = c;
    return PP_OK;
}

pp_status pp_ctx_destroy(pp_ctx* c) {
    if (!c) return PP_E_INVAL;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    drop_graphs(c);
    if (c->last_ev) (void)hipEventDestroy(c->last_ev);
    for (auto& s : c->slots)
        if (s.base && !s.external) (void)hipFree(s.base);
    if (c->plain_tab) (void)hipFree(c->plain_tab);
    if (c->batch_tab) (void)hipFree(c->batch_tab);
    if (c->debug_scratch) (void)hipFree(c->debug_scratch);
    if (c->region_scratch) (void)hipFree(c->region_scratch);
    if (c->seg_scratch) (void)hipFree(c->seg_scratch);
    for (int i = 0; i < pp_ctx::kRing; ++i) {
        if (c->staging[i]) (void)hipHostFree(c->staging[i]);
        if (c->staging_ev[i]) (void)hipEventDestroy(c->staging_ev[i]);
    }
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (int k = 0; k < pp_ctx::kMaxChains; ++k) {
        if (c->chain_stream[k]) (void)hipStreamDestroy(c->chain_stream[k]);
        if (c->join_ev[k]) (void)hipEventDestroy(c->join_ev[k]);
    }
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    for (int r = 0; r < ppk::kMaxRounds; ++r)
        for (int k = 0; k < 2; ++k)
            if (c->score_ev[r][k]) (void)hipEventDestroy(c->score_ev[r][k]);
    for (int k = 0; k < 4; ++k)
        if (c->stage_ev[k]) (void)hipEventDestroy(c->stage_ev[k]);
    delete c;
    return PP_OK;
}

// ------------------------------------------------------------------ tuning
pp_status pp_tuning_space(int32_t* n_tiles, int32_t* max_t, int32_t* n_hb, int32_t* n_chunk) {
    if (n_tiles) *n_tiles = ppk::kNumTiles;
    if (max_t) *max_t = ppk::kMaxT;
    if (n_hb) *n_hb = ppk::kNumHB;
    if (n_chunk) *n_chunk = ppk::kNumChunk;
    return PP_OK;
}

pp_status pp_set_tuning(pp_ctx* c, const pp_tuning* t) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (!t) {
        c->tuning = kDefaultTuning;
        return PP_OK;
    }
    ppk::Tuning n = c->tuning;
    if (t->diffuse_tile) {
        if (t->diffuse_tile < 1 || t->diffuse_tile > ppk::kNumTiles) return fail(c, PP_E_INVAL, "diffuse_tile out of range");
        n.diffuse_tile = t->diffuse_tile - 1;
    }
    if (t->diffuse_t) {
        if (!ppk::t_supported(t->diffuse_t)) return fail(c, PP_E_INVAL, "diffuse_t must be one of 1,2,3,4,5,8,10");
        n.diffuse_t = t->diffuse_t;
    }
    if (t->score_hb) {
        if (t->score_hb < 1 || t->score_hb > ppk::kNumHB) return fail(c, PP_E_INVAL, "score_hb out of range");
        n.score_hb = t->score_hb - 1;
    }
    if (t->score_chunk) {
        if (t->score_chunk < 1 || t->score_chunk > ppk::kNumChunk) return fail(c, PP_E_INVAL, "score_chunk out of range");
        n.score_chunk = t->score_chunk - 1;
    }
    c->tuning = n;
    drop_graphs(c);  // captured launch shapes change
    return PP_OK;
}

pp_status pp_get_tuning(const pp_ctx* c, pp_tuning* out) {
    if (!c || !out) return PP_E_INVAL;
    out->diffuse_tile = c->tuning.diffuse_tile + 1;
    out->diffuse_t = c->tuning.diffuse_t;
    out->score_hb = c->tuning.score_hb + 1;
    out->score_chunk = c->tuning.score_chunk + 1;
    return PP_OK;
}

pp_status pp_set_stage_timing(pp_ctx* c, int32_t enable) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if ((s = set_device(c)) != PP_OK) return s;
    if (enable && !c->score_ev[0][0]) {
        for (int r = 0; r < ppk::kMaxRounds; ++r)
            for (int k = 0; k < 2; ++k) HIPCHK(c, hipEventCreate(&c->score_ev[r][k]));
        for (int k = 0; k < 4; ++k) HIPCHK(c, hipEventCreate(&c->stage_ev[k]));
    }
    c->stages_valid = false;
    c->timing = enable != 0;
    c->timed_rounds = 0;
    return PP_OK;
}

pp_status pp_stage_breakdown(pp_ctx* c, float out_ms[4]) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (!out_ms) return fail(c, PP_E_INVAL, "pp_stage_breakdown: null output");
    if (!c->stages_valid) return fail(c, PP_E_INVAL, "pp_stage_breakdown: no timed batch run yet");
    float d = 0.f, n = 0.f, rr = 0.f, sc = 0.f;
    HIPCHK(c, hipEventElapsedTime(&d, c->stage_ev[0], c->stage_ev[1]));
    HIPCHK(c, hipEventElapsedTime(&n, c->stage_ev[1], c->stage_ev[2]));
    HIPCHK(c, hipEventElapsedTime(&rr, c->stage_ev[2], c->stage_ev[3]));
    for (int r = 0; r < c->timed_rounds; ++r) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->score_ev[r][0], c->score_ev[r][1]));
        sc += ms;
    }
    out_ms[0] = d;
    out_ms[1] = n;
    out_ms[2] = sc;
    out_ms[3] = rr - sc;
    return PP_OK;
}

pp_status pp_stage_time(pp_ctx* c, float* total_ms, int32_t* launches) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (!total_ms || !launches) return fail(c, PP_E_INVAL, "pp_stage_time: null output");
    float tot = 0.f;
    for (int r = 0; r < c->timed_rounds; ++r) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->score_ev[r][0], c->score_ev[r][1]));
        tot += ms;
    }
    *total_ms = tot;
    *launches = c->timed_rounds;
    return PP_OK;
}

// ------------------------------------------------------------------ stages
pp_status pp_diffuse(pp_ctx* c, const uint16_t* depth_dev, float* out_mm_dev, pp_frame_desc desc,
                     const pp_diffuse_params* p, void* stream) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (!depth_dev || !out_mm_dev || !desc_ok(desc) || !diffuse_params_ok(p))
        return fail(c, PP_E_INVAL, "pp_diffuse: bad argument");
    if ((s = set_device(c)) != PP_OK) return s;
    const size_t px = (size_t)desc.width * desc.height;
    if ((s = ensure_slot(c, 0, ppk::scan_pixels(desc.width, desc.height), 1)) != PP_OK) return s;
    FrameDev f{};
    bind_slot(c, 0, f);
    fill_geometry(f, desc);
    fill_diffuse(f, *p);
    f.depth = depth_dev;
    f.dmm = out_mm_dev;
    hipStream_t st = (hipStream_t)stream;
    if ((s = put_plain(c, f, st)) != PP_OK) return s;
    HIPCHK(c, ppk::launch_diffuse(c->plain_tab, 1, desc.width, desc.height, p->iters, p->scheme, c->tuning, st));
    return mark_stream(c, st);
}

pp_status pp_normals(pp_ctx* c, const float* depth_mm_dev, pp_frame_desc desc, pp_intrinsics K, float* points_dev,
                     float* normals_dev, uint8_t* valid_dev, void* stream) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (!depth_mm_dev || !points_dev || !normals_dev || !valid_dev || !desc_ok(desc) || !intrinsics_ok(K))
        return fail(c, PP_E_INVAL, "pp_normals: bad argument");
    if ((s = set_device(c)) != PP_OK) return s;
    FrameDev f{};
    fill_geometry(f, desc);
    f.dmm = const_cast<float*>(depth_mm_dev);
    f.pts = points_dev;
    f.nrm = normals_dev;
    f.valid = valid_dev;
    f.fx = K.fx; f.fy = K.fy; f.cx = K.cx; f.cy = K.cy;
    f.ifx = 1.0f / K.fx; f.ify = 1.0f / K.fy;
    hipStream_t st = (hipStream_t)stream;
    if ((s = put_plain(c, f, st)) != PP_OK) return s;
    HIPCHK(c, ppk::launch_normals(c->plain_tab, 1, desc.width * desc.height, false, st));
    return mark_stream(c, st);
}

static pp_status ransac_common(pp_ctx* c, const float* points_dev, const uint8_t* valid_dev, pp_frame_desc desc,
                               const pp_ransac_params* p, pp_plane* planes_dev, int32_t* n_planes_dev,
                               int8_t* labels_dev, const pp_ransac_debug* dbg, void* stream) {
    pp_status s;
    if ((s = set_device(c)) != PP_OK) return s;
    const size_t px = (size_t)desc.width * desc.height;
    if ((s = ensure_slot(c, 0, ppk::scan_pixels(desc.width, desc.height), p->hyps_per_plane)) != PP_OK) return s;
    FrameDev f{};
    bind_slot(c, 0, f);
    fill_geometry(f, desc);
    fill_ransac(f, *p);
    f.pts = const_cast<float*>(points_dev);
    f.valid = const_cast<uint8_t*>(valid_dev);
    f.labels = labels_dev;
    f.planes = planes_dev;
    f.n_planes = n_planes_dev;
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_streams(c, st)) != PP_OK) return s;
    if (dbg) {
        f.dbg = *dbg;
        if (dbg->round_info) HIPCHK(c, hipMemsetAsync(dbg->round_info, 0xFF, sizeof(int32_t) * 4 * p->max_planes, st));
    }
    if ((s = put_plain(c, f, st)) != PP_OK) return s;
    HIPCHK(c, ppk::launch_valid_list(c->plain_tab, 1, (int)px, desc.width, desc.height, false, st));
    for (int r = 0; r < p->max_planes; ++r)
        HIPCHK(c, ppk::launch_round(c->plain_tab, 1, r, (int)ppk::scan_pixels(desc.width, desc.height), p->hyps_per_plane, p->precision, c->tuning, st,
                                    c->timing ? c->score_ev[r][0] : nullptr, c->timing ? c->score_ev[r][1] : nullptr));
    if (c->timing) c->timed_rounds = p->max_planes;
    return mark_stream(c, st);
}

namespace {

// Region mode: one frame, kernels of pp_regions.hip on library scratch that
// grows on first use per shape.
pp_status regions_common(pp_ctx* c, const float* points_dev, const uint8_t* valid_dev, const int16_t* region_dev,
                         const pp_frame_desc& desc, const pp_ransac_params* p, pp_plane* planes_dev,
                         int32_t* n_planes_dev, int8_t* labels_dev, const pp_region_debug* dbg, void* stream) {
    if (p->precision != PP_SCORE_FP32)
        return fail(c, PP_E_UNSUPPORTED, "region mode scores with the FP32 residual only");
    pp_status s = set_device(c);
    if (s != PP_OK) return s;
    ppk::RegionDev r{};
    r.pts = points_dev;
    r.valid = valid_dev;
    r.region = region_dev;
    r.W = desc.width;
    r.H = desc.height;
    r.pitch = desc.pitch_px;
    r.R = p->max_planes;
    r.hyps = p->hyps_per_plane;
    r.thresh = p->thresh_m;
    r.seed = p->seed;
    r.frame_id = p->frame_id;
    r.planes = planes_dev;
    r.n_planes = n_planes_dev;
    r.labels = labels_dev;
    const size_t need = ppk::region_scratch_bytes(r.W, r.H, r.R, r.hyps);
    if (c->region_scratch_bytes < need) {
        if (c->region_scratch) {
            HIPCHK(c, hipDeviceSynchronize());
            HIPCHK(c, hipFree(c->region_scratch));
            c->region_scratch = nullptr;
            c->region_scratch_bytes = 0;
        }
        HIPCHK(c, hipMalloc(&c->region_scratch, need));
        c->region_scratch_bytes = need;
    }
    ppk::region_bind_scratch(r, c->region_scratch);
    hipStream_t st = (hipStream_t)stream;
    if ((s = order_streams(c, st)) != PP_OK) return s;
    HIPCHK(c, ppk::launch_regions(r, st));
    if (dbg) {
        const size_t R = r.R, rh = (size_t)r.R * r.hyps;
        if (dbg->npts) HIPCHK(c, hipMemcpyAsync(dbg->npts, r.npts, R * 4, hipMemcpyDeviceToDevice, st));
        if (dbg->triples)
            HIPCHK(c, hipMemcpyAsync(dbg->triples, r.triples, rh * 12, hipMemcpyDeviceToDevice, st));
        if (dbg->hyps) HIPCHK(c, hipMemcpyAsync(dbg->hyps, r.hyp, rh * 16, hipMemcpyDeviceToDevice, st));
        if (dbg->errors) HIPCHK(c, hipMemcpyAsync(dbg->errors, r.errors, rh * 8, hipMemcpyDeviceToDevice, st));
        if (dbg->counts) HIPCHK(c, hipMemcpyAsync(dbg->counts, r.counts, rh * 4, hipMemcpyDeviceToDevice, st));
        if (dbg->jstar) HIPCHK(c, hipMemcpyAsync(dbg->jstar, r.jstar, R * 4, hipMemcpyDeviceToDevice, st));
    }
    return mark_stream(c, st);
}

}  // namespace

pp_status pp_ransac_planes(pp_ctx* c, const float* points_dev, const uint8_t* valid_dev,
                           const int16_t* region_dev_or_null, pp_frame_desc desc, const pp_ransac_params* p,
                           pp_plane* planes_dev, int32_t* n_planes_dev, int8_t* labels_dev, void* stream) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (!points_dev || !valid_dev || !planes_dev || !n_planes_dev || !labels_dev || !desc_ok(desc) ||
        !ransac_params_ok(p))
        return fail(c, PP_E_INVAL, "pp_ransac_planes: bad argument");
    if (region_dev_or_null)
        return regions_common(c, points_dev, valid_dev, region_dev_or_null, desc, p, planes_dev, n_planes_dev,
                              labels_dev, nullptr, stream);
    return ransac_common(c, points_dev, valid_dev, desc, p, planes_dev, n_planes_dev, labels_dev, nullptr, stream);
}

pp_status pp_segment(pp_ctx* c, const float* normals_dev, const uint8_t* valid_dev, pp_frame_desc desc,
                     const pp_segment_params* p, int16_t* region_dev, int32_t* n_regions_dev, uint8_t* edges_dev,
                     void* stream) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (!normals_dev || !valid_dev || !region_dev || !n_regions_dev || !desc_ok(desc) || !p)
        return fail(c, PP_E_INVAL, "pp_segment: bad argument");
    if (!(p->low >= 0.f) || !(p->high >= p->low) || !isfinite(p->high) || p->max_regions < 1 ||
        p->max_regions > 32767 || p->min_area < 1 ||
        (int64_t)desc.width * desc.height > (int64_t)p->min_area * ppk::kSegMaxCand)
        return fail(c, PP_E_INVAL, "pp_segment: bad parameters");
    if ((s = set_device(c)) != PP_OK) return s;
    ppk::SegDev g{};
    g.nrm = normals_dev;
    g.valid = valid_dev;
    g.W = desc.width;
    g.H = desc.height;
    g.pitch = desc.pitch_px;
    g.min_area = p->min_area;
    g.max_regions = p->max_regions;
    g.low = p->low;
    g.high = p->high;
    g.region = region_dev;
    g.n_regions = n_regions_dev;
    g.edges = edges_dev;
    const size_t need = ppk::seg_scratch_bytes(g.W, g.H);
    if (c->seg_scratch_bytes < need) {
        if (c->seg_scratch) {
            HIPCHK(c, hipDeviceSynchronize());
            HIPCHK(c, hipFree(c->seg_scratch));
            c->seg_scratch = nullptr;
            c->seg_scratch_bytes = 0;
        }
        HIPCHK(c, hipMalloc(&c->seg_scratch, need));
        c->seg_scratch_bytes = need;
    }
    ppk::seg_bind_scratch(g, c->seg_scratch);
    if ((s = order_streams(c, (hipStream_t)stream)) != PP_OK) return s;
    HIPCHK(c, ppk::launch_segment(g, (hipStream_t)stream));
    return mark_stream(c, (hipStream_t)stream);
}

pp_status pp_ransac_regions_dbg(pp_ctx* c, const float* points_dev, const uint8_t* valid_dev,
                                const int16_t* region_dev, pp_frame_desc desc, const pp_ransac_params* p,
                                pp_plane* planes_dev, int32_t* n_planes_dev, int8_t* labels_dev,
                                const pp_region_debug* dbg, void* stream) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (!points_dev || !valid_dev || !region_dev || !planes_dev || !n_planes_dev || !labels_dev ||
        !desc_ok(desc) || !ransac_params_ok(p) || !dbg)
        return fail(c, PP_E_INVAL, "pp_ransac_regions_dbg: bad argument");
    return regions_common(c, points_dev, valid_dev, region_dev, desc, p, planes_dev, n_planes_dev, labels_dev, dbg,
                          stream);
}

pp_status pp_ransac_planes_dbg(pp_ctx* c, const float* points_dev, const uint8_t* valid_dev, pp_frame_desc desc,
                               const pp_ransac_params* p, pp_plane* planes_dev, int32_t* n_planes_dev,
                               int8_t* labels_dev, const pp_ransac_debug* dbg, void* stream) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (!points_dev || !valid_dev || !planes_dev || !n_planes_dev || !labels_dev || !desc_ok(desc) ||
        !ransac_params_ok(p) || !dbg)
        return fail(c, PP_E_INVAL, "pp_ransac_planes_dbg: bad argument");
    return ransac_common(c, points_dev, valid_dev, desc, p, planes_dev, n_planes_dev, labels_dev, dbg, stream);
}

pp_status pp_debug_score_triples(pp_ctx* c, const float* points_dev, const uint8_t* valid_dev, pp_frame_desc desc,
                                 const int32_t* triples_dev, int32_t n, float thresh_m, int32_t precision,
                                 float recheck_band_m, float* planes_dev, int32_t* counts_dev, void* stream) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (!points_dev || !valid_dev || !triples_dev || !planes_dev || !counts_dev || !desc_ok(desc) || n < 1 ||
        n > (1 << 24) || !(thresh_m > 0.f) || precision < PP_SCORE_FP32 || precision > PP_SCORE_FP16 ||
        !(recheck_band_m >= 0.f))
        return fail(c, PP_E_INVAL, "pp_debug_score_triples: bad argument");
    if ((s = set_device(c)) != PP_OK) return s;
    const size_t px = (size_t)desc.width * desc.height;
    if ((s = ensure_slot(c, 0, ppk::scan_pixels(desc.width, desc.height), 1)) != PP_OK) return s;
    FrameDev f{};
    bind_slot(c, 0, f);
    fill_geometry(f, desc);
    f.pts = const_cast<float*>(points_dev);
    f.valid = const_cast<uint8_t*>(valid_dev);
    f.thresh = thresh_m;
    f.band = recheck_band_m;
    f.precision = precision;
    f.max_planes = 1;
    f.hyps = n;
    f.hyp = reinterpret_cast<float4*>(planes_dev);
    f.counts = counts_dev;
    // the valid-list pass writes labels and n_planes; point them at scratch
    const size_t need = align256(px) + 256;
    if (c->debug_scratch_bytes < need) {
        if (c->debug_scratch) {
            HIPCHK(c, hipDeviceSynchronize());
            HIPCHK(c, hipFree(c->debug_scratch));
            c->debug_scratch = nullptr;
            c->debug_scratch_bytes = 0;
        }
        HIPCHK(c, hipMalloc(&c->debug_scratch, need));
        c->debug_scratch_bytes = need;
    }
    f.labels = static_cast<int8_t*>(c->debug_scratch);
    f.n_planes = reinterpret_cast<int32_t*>(static_cast<char*>(c->debug_scratch) + align256(px));
    hipStream_t st = (hipStream_t)stream;
    if ((s = put_plain(c, f, st)) != PP_OK) return s;
    HIPCHK(c, ppk::launch_valid_list(c->plain_tab, 1, (int)px, desc.width, desc.height, false, st));
    hipLaunchKernelGGL(k_force_active, dim3(1), dim3(1), 0, st, c->plain_tab);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, ppk::launch_hyp_from_triples(c->plain_tab, triples_dev, n, st));
    HIPCHK(c, ppk::launch_score_only(c->plain_tab, (int)ppk::scan_pixels(desc.width, desc.height), n, precision, c->tuning, st));
    return mark_stream(c, st);
}

}  // extern "C"

// ------------------------------------------------------------------ batches
namespace {

bool job_ok(const pp_frame_job& j) {
    return j.depth && j.depth_mm && j.points && j.normals && j.valid && j.planes && j.n_planes && j.labels &&
           desc_ok(j.desc) && intrinsics_ok(j.K) && diffuse_params_ok(&j.diffuse) && ransac_params_ok(&j.ransac);
}

struct BatchPlan {
    int nf = 0, maxW = 0, maxH = 0, max_px = 0, max_scan = 0, max_hyps = 0, max_rounds = 0, precision = 0;
    std::vector<int> order;                        // table position -> job index
    std::vector<std::pair<int, int>> iter_groups;  // (first table position, count): equal iterations and scheme
    std::vector<int> group_iters, group_scheme;
    std::string key;
};

BatchPlan plan_batch(const pp_frame_job* jobs, int n, const ppk::Tuning& tu) {
    BatchPlan b;
    b.nf = n;
    b.precision = jobs[0].ransac.precision;
    b.order.resize(n);
    for (int i = 0; i < n; ++i) b.order[i] = i;
    std::stable_sort(b.order.begin(), b.order.end(), [&](int a, int c) {
        const pp_diffuse_params &pa = jobs[a].diffuse, &pc = jobs[c].diffuse;
        return pa.scheme != pc.scheme ? pa.scheme < pc.scheme : pa.iters < pc.iters;
    });
    for (int i = 0; i < n; ++i) {
        const pp_frame_job& j = jobs[b.order[i]];
        b.maxW = std::max(b.maxW, j.desc.width);
        b.maxH = std::max(b.maxH, j.desc.height);
        b.max_px = std::max(b.max_px, j.desc.width * j.desc.height);
        b.max_scan = std::max(b.max_scan, (int)ppk::scan_pixels(j.desc.width, j.desc.height));
        b.max_hyps = std::max(b.max_hyps, j.ransac.hyps_per_plane);
        b.max_rounds = std::max(b.max_rounds, j.ransac.max_planes);
        if (i == 0 || j.diffuse.iters != jobs[b.order[i - 1]].diffuse.iters ||
            j.diffuse.scheme != jobs[b.order[i - 1]].diffuse.scheme) {
            b.iter_groups.push_back({i, 0});
            b.group_iters.push_back(j.diffuse.iters);
            b.group_scheme.push_back(j.diffuse.scheme);
        }
        b.iter_groups.back().second++;
    }
    char buf[256];
    snprintf(buf, sizeof buf, "n%d W%d H%d px%d q%d h%d r%d p%d t%d.%d.%d.%d", n, b.maxW, b.maxH, b.max_px, b.max_scan,
             b.max_hyps, b.max_rounds, b.precision, tu.diffuse_tile, tu.diffuse_t, tu.score_hb, tu.score_chunk);
    b.key = buf;
    for (size_t g = 0; g < b.iter_groups.size(); ++g) {
        snprintf(buf, sizeof buf, " g%d:%d:%d:%d", b.iter_groups[g].first, b.iter_groups[g].second, b.group_iters[g],
                 b.group_scheme[g]);
        b.key += buf;
    }
    return b;
}

// Frames per kernel chain of a batch: with several chains, one chain's
// latency-bound kernels (hypotheses, refit, removal of a few frames) overlap
// with another's scoring, where one chain would leave the GPU mostly idle
// between its launches.
constexpr int kChainFrames = 8;

// Frames [f0, f1) of the (sorted) batch table as one chain of launches on st.
pp_status enqueue_chain(pp_ctx* c, const BatchPlan& b, int f0, int f1, hipStream_t st) {
    FrameDev* tab = c->batch_tab + f0;
    const int nf = f1 - f0;
    for (size_t g = 0; g < b.iter_groups.size(); ++g) {
        const int g0 = std::max(b.iter_groups[g].first, f0);
        const int g1 = std::min(b.iter_groups[g].first + b.iter_groups[g].second, f1);
        if (g0 < g1)
            HIPCHK(c, ppk::launch_diffuse(c->batch_tab + g0, g1 - g0, b.maxW, b.maxH, b.group_iters[g], b.group_scheme[g],
                                          c->tuning, st));
    }
    HIPCHK(c, ppk::launch_normals(tab, nf, b.max_px, true, st));
    HIPCHK(c, ppk::launch_valid_list(tab, nf, b.max_px, b.maxW, b.maxH, true, st));
    for (int r = 0; r < b.max_rounds; ++r)
        HIPCHK(c, ppk::launch_round(tab, nf, r, b.max_scan, b.max_hyps, b.precision, c->tuning, st));
    return PP_OK;
}

pp_status enqueue_batch(pp_ctx* c, const BatchPlan& b, hipStream_t st, bool capturing) {
    const bool timed = c->timing && !capturing;
    const int chains = c->chains ? std::min(pp_ctx::kMaxChains, b.nf / kChainFrames) : 1;
    if (!timed && chains > 1) {
        for (int k = 1; k < chains; ++k) {
            if (!c->chain_stream[k]) HIPCHK(c, hipStreamCreateWithFlags(&c->chain_stream[k], hipStreamNonBlocking));
            if (!c->join_ev[k]) HIPCHK(c, hipEventCreateWithFlags(&c->join_ev[k], hipEventDisableTiming));
        }
        if (!c->fork_ev) HIPCHK(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
        HIPCHK(c, hipEventRecord(c->fork_ev, st));
        for (int k = 1; k < chains; ++k) HIPCHK(c, hipStreamWaitEvent(c->chain_stream[k], c->fork_ev, 0));
        pp_status s;
        for (int k = 0; k < chains; ++k) {
            const int f0 = (int)((int64_t)b.nf * k / chains), f1 = (int)((int64_t)b.nf * (k + 1) / chains);
            if ((s = enqueue_chain(c, b, f0, f1, k ? c->chain_stream[k] : st)) != PP_OK) return s;
        }
        for (int k = 1; k < chains; ++k) {
            HIPCHK(c, hipEventRecord(c->join_ev[k], c->chain_stream[k]));
            HIPCHK(c, hipStreamWaitEvent(st, c->join_ev[k], 0));
        }
        return PP_OK;
    }
    if (timed) HIPCHK(c, hipEventRecord(c->stage_ev[0], st));
    for (size_t g = 0; g < b.iter_groups.size(); ++g)
        HIPCHK(c, ppk::launch_diffuse(c->batch_tab + b.iter_groups[g].first, b.iter_groups[g].second, b.maxW, b.maxH,
                                      b.group_iters[g], b.group_scheme[g], c->tuning, st));
    if (timed) HIPCHK(c, hipEventRecord(c->stage_ev[1], st));
    HIPCHK(c, ppk::launch_normals(c->batch_tab, b.nf, b.max_px, true, st));
    HIPCHK(c, ppk::launch_valid_list(c->batch_tab, b.nf, b.max_px, b.maxW, b.maxH, true, st));
    if (timed) HIPCHK(c, hipEventRecord(c->stage_ev[2], st));
    for (int r = 0; r < b.max_rounds; ++r)
        HIPCHK(c, ppk::launch_round(c->batch_tab, b.nf, r, b.max_scan, b.max_hyps, b.precision, c->tuning, st,
                                    timed ? c->score_ev[r][0] : nullptr, timed ? c->score_ev[r][1] : nullptr));
    if (timed) {
        HIPCHK(c, hipEventRecord(c->stage_ev[3], st));
        c->timed_rounds = b.max_rounds;
        c->stages_valid = true;
    }
    return PP_OK;
}

pp_status upload_batch_table(pp_ctx* c, const pp_frame_job* jobs, const BatchPlan& b, hipStream_t st) {
    pp_status s;
    for (int i = 0; i < b.nf; ++i) {
        const pp_frame_job& j = jobs[b.order[i]];
        if ((s = ensure_slot(c, 1 + i, ppk::scan_pixels(j.desc.width, j.desc.height), j.ransac.hyps_per_plane)) != PP_OK) return s;
    }
    if (b.nf > c->batch_tab_cap) {
        if (c->batch_tab) {
            HIPCHK(c, hipDeviceSynchronize());
            HIPCHK(c, hipFree(c->batch_tab));
            c->batch_tab = nullptr;
        }
        HIPCHK(c, hipMalloc(&c->batch_tab, sizeof(FrameDev) * b.nf));
        c->batch_tab_cap = b.nf;
        drop_graphs(c);  // captured graphs reference the old table
    }
    const int k = c->ring_pos;
    c->ring_pos = (k + 1) % pp_ctx::kRing;
    if (c->staging_used[k]) HIPCHK(c, hipEventSynchronize(c->staging_ev[k]));
    if (c->staging_cap[k] < b.nf) {
        if (c->staging[k]) HIPCHK(c, hipHostFree(c->staging[k]));
        c->staging[k] = nullptr;
        HIPCHK(c, hipHostMalloc((void**)&c->staging[k], sizeof(FrameDev) * b.nf, hipHostMallocDefault));
        c->staging_cap[k] = b.nf;
    }
    for (int i = 0; i < b.nf; ++i) {
        const pp_frame_job& j = jobs[b.order[i]];
        FrameDev f{};
        bind_slot(c, 1 + i, f);
        fill_geometry(f, j.desc);
        fill_diffuse(f, j.diffuse);
        fill_ransac(f, j.ransac);
        f.fx = j.K.fx; f.fy = j.K.fy; f.cx = j.K.cx; f.cy = j.K.cy;
        f.ifx = 1.0f / j.K.fx; f.ify = 1.0f / j.K.fy;
        f.depth = j.depth;
        f.dmm = j.depth_mm;
        f.pts = j.points;
        f.nrm = j.normals;
        f.valid = j.valid;
        f.labels = j.labels;
        f.planes = j.planes;
        f.n_planes = j.n_planes;
        c->staging[k][i] = f;
    }
    HIPCHK(c, hipMemcpyAsync(c->batch_tab, c->staging[k], sizeof(FrameDev) * b.nf, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipEventRecord(c->staging_ev[k], st));
    c->staging_used[k] = true;
    return PP_OK;
}

pp_status batch_run(pp_ctx* c, int32_t n, const pp_frame_job* jobs, void* stream, bool use_graph,
                    void* const* ext_scratch = nullptr) {
    pp_status s = check_ctx(c);
    if (s != PP_OK) return s;
    if (n < 1 || n > 65535 || !jobs) return fail(c, PP_E_INVAL, "pp_batch_run: bad frame count");
    for (int i = 0; i < n; ++i) {
        if (!job_ok(jobs[i])) return fail(c, PP_E_INVAL, "pp_batch_run: bad job " + std::to_string(i));
        if (jobs[i].ransac.precision != jobs[0].ransac.precision)
            return fail(c, PP_E_INVAL, "pp_batch_run: all frames of a batch must use one scoring precision");
    }
    if ((s = set_device(c)) != PP_OK) return s;
    BatchPlan b = plan_batch(jobs, n, c->tuning);
    hipStream_t st = (hipStream_t)stream;
    if (ext_scratch) {
        if ((int)c->slots.size() < n + 1) c->slots.resize(n + 1);
        for (int i = 0; i < n; ++i) {
            const pp_frame_job& j = jobs[b.order[i]];
            Slot& sl = c->slots[1 + i];
            if (sl.base && !sl.external) {
                HIPCHK(c, hipDeviceSynchronize());
                HIPCHK(c, hipFree(sl.base));
            }
            sl.base = ext_scratch[b.order[i]];
            sl.px_cap = ppk::scan_pixels(j.desc.width, j.desc.height);
            sl.hyp_cap = j.ransac.hyps_per_plane;
            sl.bytes = slot_layout(sl.px_cap, sl.hyp_cap).total;
            sl.external = true;
        }
    }
    if ((s = order_streams(c, st)) != PP_OK) return s;
    if ((s = upload_batch_table(c, jobs, b, st)) != PP_OK) return s;
    if (!use_graph) {
        if ((s = enqueue_batch(c, b, st, false)) != PP_OK) return s;
        return mark_stream(c, st);
    }
    auto it = c->graphs.find(b.key);
    if (it == c->graphs.end()) {
        if (c->graphs.size() >= kMaxGraphs) {  // the least recently used layout goes
            auto lru = c->graphs.begin();
            for (auto g = c->graphs.begin(); g != c->graphs.end(); ++g)
                if (g->second.last_use < lru->second.last_use) lru = g;
            destroy_graph(lru->second);
            c->graphs.erase(lru);
        }
        hipGraph_t g = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
        pp_status es = enqueue_batch(c, b, c->capture_stream, true);
        hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
        if (es != PP_OK) {
            if (g) (void)hipGraphDestroy(g);
            return es;
        }
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
        GraphEntry ge;
        e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
        e = hipEventCreateWithFlags(&ge.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipGraphExecDestroy(ge.exec);
            return hip_fail(c, e, "hipEventCreateWithFlags");
        }
        it = c->graphs.emplace(b.key, ge).first;
    }
    it->second.last_use = ++c->graph_clock;
    HIPCHK(c, hipGraphLaunch(it->second.exec, st));
    HIPCHK(c, hipEventRecord(it->second.done, st));
    return mark_stream(c, st);
}

}  // namespace

extern "C" {

pp_status pp_validate_job(const pp_frame_job* job) { return job && job_ok(*job) ? PP_OK : PP_E_INVAL; }

pp_status pp_batch_run(pp_ctx* c, int32_t n, const pp_frame_job* jobs, void* stream) {
    return batch_run(c, n, jobs, stream, true);
}

pp_status pp_batch_run_eager(pp_ctx* c, int32_t n, const pp_frame_job* jobs, void* stream) {
    return batch_run(c, n, jobs, stream, false);
}

}  // extern "C"

namespace ppk {

size_t frame_scratch_bytes(int width, int height, int hyps) {
    return slot_layout(ppk::scan_pixels(width, height), hyps).total;
}

pp_status batch_run_external(pp_ctx* c, int n, const pp_frame_job* jobs, void* const* scratch, hipStream_t s,
                             bool graph) {
    // the serving runtime's batches run as one kernel chain: concurrent chains
    // are not validated inside its captured graphs
    if (c) c->chains = false;
    return batch_run(c, n, jobs, (void*)s, graph, scratch);
}

const char* ctx_error(const pp_ctx* c) { return c->last_error.c_str(); }

}  // namespace ppk

// ------------------------------------------------------------------ RANSAC without allocation
// Scratch of pp_ransac_planes_noalloc: the one-entry frame table followed by
// one frame slot (slot_layout).  Each GPU the library runs on holds its own
// copy until the process ends.  In host code the array's name stands for a
// host-side shadow, not device memory: only the per-device address that
// hipGetSymbolAddress returns is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[PP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocDevices] = {};

// Device address of `scratch` on device dev (the current device), looked up
// once per device.
pp_status noalloc_scratch(int dev, void** out) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(nullptr, PP_E_HIP,
                        std::string("pp_ransac_planes_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        }
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return PP_OK;
}

// Bytes of `scratch` one frame takes: the frame table entry, then its slot.
size_t noalloc_bytes(const pp_frame_desc& d, int hyps) {
    return align256(sizeof(FrameDev)) + slot_layout(ppk::scan_pixels(d.width, d.height), hyps).total;
}

}  // namespace

extern "C" {

pp_status pp_ransac_planes_noalloc(const float* points_dev, const uint8_t* valid_dev, pp_frame_desc desc,
                                   const pp_ransac_params* p, pp_plane* planes_dev, int32_t* n_planes_dev,
                                   int8_t* labels_dev, void* stream) {
    if (!points_dev || !valid_dev || !planes_dev || !n_planes_dev || !labels_dev || !desc_ok(desc) ||
        !ransac_params_ok(p))
        return fail(nullptr, PP_E_INVAL, "pp_ransac_planes_noalloc: bad argument");
    const size_t need = noalloc_bytes(desc, p->hyps_per_plane);
    if (need > PP_NOALLOC_SCRATCH_BYTES)
        return fail(nullptr, PP_E_INVAL,
                    "pp_ransac_planes_noalloc: the frame needs " + std::to_string(need) +
                        " bytes of scratch, more than the " + std::to_string((size_t)PP_NOALLOC_SCRATCH_BYTES) +
                        " the library holds per GPU");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kNoAllocDevices) {
        (void)hipGetLastError();
        return fail(nullptr, e != hipSuccess ? PP_E_HIP : PP_E_UNSUPPORTED,
                    "pp_ransac_planes_noalloc: no usable current device");
    }
    void* base = nullptr;
    pp_status s = noalloc_scratch(dev, &base);
    if (s != PP_OK) return s;
    FrameDev* tab = static_cast<FrameDev*>(base);
    const size_t px = (size_t)desc.width * desc.height;
    FrameDev f{};
    bind_layout(static_cast<char*>(base) + align256(sizeof(FrameDev)), ppk::scan_pixels(desc.width, desc.height), p->hyps_per_plane, f);
    fill_geometry(f, desc);
    fill_ransac(f, *p);
    f.pts = const_cast<float*>(points_dev);
    f.valid = const_cast<uint8_t*>(valid_dev);
    f.labels = labels_dev;
    f.planes = planes_dev;
    f.n_planes = n_planes_dev;
    // every scratch field the kernels read is written earlier in the same
    // call (the valid-list kernels set the round state, the per-point bytes,
    // the lists and the chunk counts), so nothing is cleared here
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_set_frame, dim3(1), dim3(1), 0, st, tab, f);
    e = hipGetLastError();
    if (e == hipSuccess) e = ppk::launch_valid_list(tab, 1, (int)px, desc.width, desc.height, false, st);
    for (int r = 0; e == hipSuccess && r < p->max_planes; ++r)
        e = ppk::launch_round(tab, 1, r, (int)ppk::scan_pixels(desc.width, desc.height), p->hyps_per_plane, p->precision, kDefaultTuning, st);
    if (e != hipSuccess) return fail(nullptr, PP_E_HIP, std::string("pp_ransac_planes_noalloc: ") + hipGetErrorString(e));
    return PP_OK;
}

}  // extern "C"
