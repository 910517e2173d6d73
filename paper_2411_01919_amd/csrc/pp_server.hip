// Serving runtime of libpp.so: several camera streams submit frames as they
// arrive; a scheduler thread admits them against an HBM budget, groups the
// admitted frames into ragged batches and launches them on one of several HIP
// streams ("lanes"), so frames that arrive while others run are admitted as
// memory frees up and overlap with them on the device (continuous batching
// at batch granularity).  Every frame's computation is independent of what it
// is batched with, so a result is bitwise the same alone and in the mix.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pp_internal.h"

namespace {

double now_us() {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

// First-fit allocator over one device allocation, free blocks coalesced.
class Arena {
public:
    void reset(size_t cap) {
        cap_ = cap;
        free_.clear();
        if (cap) free_[0] = cap;
        used_ = peak_ = 0;
    }
    bool alloc(size_t n, size_t* off) {
        n = a256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n;
            const size_t noff = it->first + n;
            free_.erase(it);
            if (rest) free_[noff] = rest;
            used_ += n;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = a256(n);
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

private:
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

enum TicketState { T_QUEUED, T_ADMITTED, T_INFLIGHT, T_DONE, T_FAILED, T_CANCELLED };

struct Ticket {
    int stream = 0;
    uint64_t frame_id = 0;
    int slot = 0;
    TicketState state = T_QUEUED;
    size_t off = 0, bytes = 0;
    double t_submit = 0.0, t_done = 0.0;
    pp_status err = PP_OK;
};

// Byte offsets of one frame's buffers inside its arena block.
struct FrameBlock {
    size_t depth, dmm, pts, nrm, valid, labels, planes, nplanes, scratch, total;
};

FrameBlock frame_block(int W, int H, int max_planes, int hyps) {
    const size_t px = (size_t)W * H;
    FrameBlock b;
    size_t o = 0;
    b.depth = o; o += a256(px * 2);
    b.dmm = o; o += a256(px * 4);
    b.pts = o; o += a256(px * 12);
    b.nrm = o; o += a256(px * 12);
    b.valid = o; o += a256(px);
    b.labels = o; o += a256(px);
    b.planes = o; o += a256((size_t)max_planes * sizeof(pp_plane));
    b.nplanes = o; o += 256;
    b.scratch = o; o += a256(ppk::frame_scratch_bytes(W, H, hyps));
    b.total = o;
    return b;
}

struct Stream {
    pp_frame_desc desc{};
    pp_intrinsics K{};
    pp_diffuse_params dp{};
    pp_ransac_params rp{};
    FrameBlock blk{};
    size_t in_bytes = 0, out_bytes = 0;  // per staging slot
    char* in_stage = nullptr;            // pinned [slots][in_bytes]
    char* out_stage = nullptr;           // pinned [slots][out_bytes]: planes, n_planes, labels
    std::vector<int> free_slots;
    int outstanding = 0;
    bool open = true;
};

struct Lane {
    hipStream_t stream = nullptr;
    pp_ctx* ctx = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    bool dry_fail = false;  // dry run: this batch ends as a failed HIP batch would
    double dry_done_at = 0.0;
    std::vector<uint64_t> tickets;
};

}  // namespace

struct pp_server {
    pp_server_cfg cfg{};
    bool dry = false;
    void* arena_base = nullptr;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread thr;
    bool stop = false;
    bool poisoned = false;
    std::string err;
    std::map<int, Stream> streams;
    std::unordered_map<uint64_t, Ticket> tickets;
    std::deque<uint64_t> queue;  // T_QUEUED, arrival order
    std::deque<uint64_t> ready;  // T_ADMITTED, waiting for a lane
    std::vector<Lane> lanes;
    uint64_t seq = 0;
    // statistics
    uint64_t submitted = 0, completed = 0, rejected = 0, cancelled = 0, launches = 0, launched_frames = 0;
    std::vector<double> lat;
    size_t lat_pos = 0;
};

namespace {

constexpr size_t kLatWindow = 65536;

void record_latency(pp_server* s, double us) {
    if (s->lat.size() < kLatWindow)
        s->lat.push_back(us);
    else
        s->lat[s->lat_pos++ % kLatWindow] = us;
}

pp_status poison(pp_server* s, const std::string& msg) {
    s->poisoned = true;
    s->err = msg;
    for (auto& kv : s->tickets)
        if (kv.second.state == T_QUEUED || kv.second.state == T_ADMITTED || kv.second.state == T_INFLIGHT) {
            kv.second.state = T_FAILED;
            kv.second.err = PP_E_HIP;
        }
    s->queue.clear();
    s->ready.clear();
    s->cv_done.notify_all();
    return PP_E_HIP;
}

void release_frame(pp_server* s, Ticket& t) {
    if (t.bytes) s->arena.release(t.off, t.bytes);
    t.bytes = 0;
}

// Completion of a lane's batch: tickets become pollable, memory is freed.
void finish_lane(pp_server* s, Lane& L) {
    const double t = now_us();
    for (uint64_t id : L.tickets) {
        auto it = s->tickets.find(id);
        if (it == s->tickets.end()) continue;
        Ticket& tk = it->second;
        release_frame(s, tk);
        if (tk.state != T_INFLIGHT) continue;
        tk.state = T_DONE;
        tk.t_done = t;
        ++s->completed;
        record_latency(s, t - tk.t_submit);
    }
    L.tickets.clear();
    L.busy = false;
    s->cv_done.notify_all();
}

void poll_lanes(pp_server* s) {
    for (auto& L : s->lanes) {
        if (!L.busy) continue;
        if (s->dry) {
            if (now_us() < L.dry_done_at) continue;
            if (L.dry_fail) {
                L.dry_fail = false;
                L.busy = false;
                L.tickets.clear();
                poison(s, "batch failed: injected failure (dry run)");
            } else {
                finish_lane(s, L);
            }
            continue;
        }
        const hipError_t e = hipEventQuery(L.done);
        if (e == hipSuccess)
            finish_lane(s, L);
        else if (e != hipErrorNotReady) {
            poison(s, std::string("batch failed: ") + hipGetErrorString(e));
            L.busy = false;
            L.tickets.clear();
        }
    }
}

// Admission in arrival order: a frame is admitted once its block fits.
void admit(pp_server* s) {
    while (!s->queue.empty()) {
        const uint64_t id = s->queue.front();
        Ticket& t = s->tickets[id];
        const Stream& st = s->streams[t.stream];
        size_t off = 0;
        if (!s->arena.alloc(st.blk.total, &off)) break;
        t.off = off;
        t.bytes = st.blk.total;
        t.state = T_ADMITTED;
        s->queue.pop_front();
        s->ready.push_back(id);
    }
}

pp_status launch_on(pp_server* s, Lane& L) {
    // one scoring precision per batch: take the oldest ready frame's, then others that match
    std::vector<uint64_t> take;
    const int prec = s->streams[s->tickets[s->ready.front()].stream].rp.precision;
    for (auto it = s->ready.begin(); it != s->ready.end() && (int)take.size() < s->cfg.max_batch;) {
        if (s->streams[s->tickets[*it].stream].rp.precision == prec) {
            take.push_back(*it);
            it = s->ready.erase(it);
        } else {
            ++it;
        }
    }
    for (uint64_t id : take) s->tickets[id].state = T_INFLIGHT;
    L.tickets = take;
    L.busy = true;
    ++s->launches;
    s->launched_frames += take.size();
    if (s->dry) {
        L.dry_done_at = now_us() + s->cfg.dry_run_us;
        L.dry_fail = s->cfg.dry_run_fail_batch > 0 && s->launches == (uint64_t)s->cfg.dry_run_fail_batch;
        return PP_OK;
    }
    char* base = static_cast<char*>(s->arena_base);
    std::vector<pp_frame_job> jobs(take.size());
    std::vector<void*> scratch(take.size());
    for (size_t i = 0; i < take.size(); ++i) {
        Ticket& t = s->tickets[take[i]];
        Stream& st = s->streams[t.stream];
        char* fb = base + t.off;
        const size_t px = (size_t)st.desc.width * st.desc.height;
        hipError_t e = hipMemcpyAsync(fb + st.blk.depth, st.in_stage + (size_t)t.slot * st.in_bytes, px * 2,
                                      hipMemcpyHostToDevice, L.stream);
        if (e != hipSuccess) return poison(s, std::string("input copy: ") + hipGetErrorString(e));
        pp_frame_job& j = jobs[i];
        j.depth = reinterpret_cast<const uint16_t*>(fb + st.blk.depth);
        j.desc = st.desc;
        j.K = st.K;
        j.diffuse = st.dp;
        j.ransac = st.rp;
        j.ransac.frame_id = t.frame_id;
        j.depth_mm = reinterpret_cast<float*>(fb + st.blk.dmm);
        j.points = reinterpret_cast<float*>(fb + st.blk.pts);
        j.normals = reinterpret_cast<float*>(fb + st.blk.nrm);
        j.valid = reinterpret_cast<uint8_t*>(fb + st.blk.valid);
        j.labels = reinterpret_cast<int8_t*>(fb + st.blk.labels);
        j.planes = reinterpret_cast<pp_plane*>(fb + st.blk.planes);
        j.n_planes = reinterpret_cast<int32_t*>(fb + st.blk.nplanes);
        scratch[i] = fb + st.blk.scratch;
    }
    pp_status ps = ppk::batch_run_external(L.ctx, (int)jobs.size(), jobs.data(), scratch.data(), L.stream,
                                           s->cfg.use_graphs != 0);
    if (ps != PP_OK) return poison(s, std::string("batch launch: ") + ppk::ctx_error(L.ctx));
    for (size_t i = 0; i < take.size(); ++i) {
        Ticket& t = s->tickets[take[i]];
        Stream& st = s->streams[t.stream];
        char* fb = base + t.off;
        char* out = st.out_stage + (size_t)t.slot * st.out_bytes;
        const size_t pb = (size_t)st.rp.max_planes * sizeof(pp_plane);
        const size_t px = (size_t)st.desc.width * st.desc.height;
        hipError_t e = hipMemcpyAsync(out, fb + st.blk.planes, pb, hipMemcpyDeviceToHost, L.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(out + pb, fb + st.blk.nplanes, 4, hipMemcpyDeviceToHost, L.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(out + pb + 256, fb + st.blk.labels, px, hipMemcpyDeviceToHost, L.stream);
        if (e != hipSuccess) return poison(s, std::string("result copy: ") + hipGetErrorString(e));
    }
    const hipError_t e = hipEventRecord(L.done, L.stream);
    if (e != hipSuccess) return poison(s, std::string("event: ") + hipGetErrorString(e));
    return PP_OK;
}

void scheduler(pp_server* s) {
    if (!s->dry) (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        poll_lanes(s);
        if (!s->poisoned) {
            admit(s);
            for (auto& L : s->lanes) {
                if (s->ready.empty() || s->poisoned) break;
                if (!L.busy) launch_on(s, L);
            }
        }
        bool busy = false;
        for (auto& L : s->lanes) busy = busy || L.busy;
        // with work on the device, wake often to notice completions; otherwise wait for submissions
        s->cv_work.wait_for(lk, std::chrono::microseconds(busy ? 20 : 2000));
    }
}

pp_status check(pp_server* s) {
    if (!s) return PP_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    return s->poisoned ? PP_E_HIP : PP_OK;
}

}  // namespace

extern "C" {

pp_status pp_server_create(const pp_server_cfg* cfg, pp_server** out) {
    if (!cfg || !out || cfg->hbm_budget_bytes < (1u << 20) || cfg->max_batch < 1 || cfg->max_batch > 1024 ||
        cfg->lanes < 1 || cfg->lanes > 4 || cfg->staging_frames < 1 || cfg->staging_frames > 1024 ||
        cfg->dry_run_us < 0 || cfg->dry_run_fail_batch < 0 || (cfg->dry_run_fail_batch > 0 && cfg->dry_run_us == 0))
        return PP_E_INVAL;
    *out = nullptr;
    pp_server* s = new pp_server();
    s->cfg = *cfg;
    s->dry = cfg->dry_run_us > 0;
    s->lanes.resize(cfg->lanes);
    if (!s->dry) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || n <= cfg->device || cfg->device < 0) {
            (void)hipGetLastError();
            delete s;
            return PP_E_NODEVICE;
        }
        hipError_t e = hipSetDevice(cfg->device);
        if (e == hipSuccess) e = hipMalloc(&s->arena_base, cfg->hbm_budget_bytes);
        for (auto& L : s->lanes) {
            if (e != hipSuccess) break;
            e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
            if (e == hipSuccess && pp_ctx_create(cfg->device, &L.ctx) != PP_OK) e = hipErrorOutOfMemory;
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            pp_server_destroy(s);
            return e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation ? PP_E_NOMEM : PP_E_HIP;
        }
    }
    s->arena.reset(cfg->hbm_budget_bytes);
    s->thr = std::thread(scheduler, s);
    *out = s;
    return PP_OK;
}

pp_status pp_server_destroy(pp_server* s) {
    if (!s) return PP_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->thr.joinable()) s->thr.join();
    if (!s->dry) {
        (void)hipSetDevice(s->cfg.device);
        for (auto& L : s->lanes) {
            if (L.stream) (void)hipStreamSynchronize(L.stream);
            if (L.ctx) pp_ctx_destroy(L.ctx);
            if (L.done) (void)hipEventDestroy(L.done);
            if (L.stream) (void)hipStreamDestroy(L.stream);
        }
        for (auto& kv : s->streams) {
            if (kv.second.in_stage) (void)hipHostFree(kv.second.in_stage);
            if (kv.second.out_stage) (void)hipHostFree(kv.second.out_stage);
        }
        if (s->arena_base) (void)hipFree(s->arena_base);
    } else {
        for (auto& kv : s->streams) {
            free(kv.second.in_stage);
            free(kv.second.out_stage);
        }
    }
    delete s;
    return PP_OK;
}

const char* pp_server_last_error(const pp_server* s) {
    // a copy per calling thread: the scheduler may replace the text meanwhile
    thread_local std::string text;
    if (!s) return "";
    std::lock_guard<std::mutex> lk(const_cast<pp_server*>(s)->mu);
    text = s->err;
    return text.c_str();
}

pp_status pp_stream_open(pp_server* s, int32_t stream_id, pp_frame_desc desc, pp_intrinsics K,
                         const pp_diffuse_params* dp, const pp_ransac_params* rp) {
    pp_status c = check(s);
    if (c != PP_OK) return c;
    pp_frame_job probe{};
    probe.depth = reinterpret_cast<const uint16_t*>(1);
    probe.depth_mm = probe.points = probe.normals = reinterpret_cast<float*>(1);
    probe.valid = reinterpret_cast<uint8_t*>(1);
    probe.planes = reinterpret_cast<pp_plane*>(1);
    probe.n_planes = reinterpret_cast<int32_t*>(1);
    probe.labels = reinterpret_cast<int8_t*>(1);
    probe.desc = desc;
    probe.K = K;
    if (!dp || !rp) return PP_E_INVAL;
    probe.diffuse = *dp;
    probe.ransac = *rp;
    if (desc.pitch_px != desc.width || pp_validate_job(&probe) != PP_OK) return PP_E_INVAL;
    Stream st;
    st.desc = desc;
    st.K = K;
    st.dp = *dp;
    st.rp = *rp;
    st.blk = frame_block(desc.width, desc.height, rp->max_planes, rp->hyps_per_plane);
    if (st.blk.total > s->cfg.hbm_budget_bytes) return PP_E_BUDGET;  // a frame of this stream can never fit
    const size_t px = (size_t)desc.width * desc.height;
    st.in_bytes = a256(px * 2);
    st.out_bytes = a256((size_t)rp->max_planes * sizeof(pp_plane)) + 256 + a256(px);
    const size_t n = (size_t)s->cfg.staging_frames;
    if (s->dry) {
        st.in_stage = static_cast<char*>(malloc(n * st.in_bytes));
        st.out_stage = static_cast<char*>(calloc(n, st.out_bytes));
        if (!st.in_stage || !st.out_stage) {
            free(st.in_stage);
            free(st.out_stage);
            return PP_E_NOMEM;
        }
    } else {
        (void)hipSetDevice(s->cfg.device);
        if (hipHostMalloc((void**)&st.in_stage, n * st.in_bytes, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&st.out_stage, n * st.out_bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            if (st.in_stage) (void)hipHostFree(st.in_stage);
            return PP_E_NOMEM;
        }
    }
    for (int i = (int)n - 1; i >= 0; --i) st.free_slots.push_back(i);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->streams.count(stream_id)) {
        if (s->dry) {
            free(st.in_stage);
            free(st.out_stage);
        } else {
            (void)hipHostFree(st.in_stage);
            (void)hipHostFree(st.out_stage);
        }
        return PP_E_INVAL;  // ids are unique for the server's lifetime
    }
    s->streams.emplace(stream_id, std::move(st));
    return PP_OK;
}

pp_status pp_stream_close(pp_server* s, int32_t stream_id) {
    if (!s) return PP_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->streams.find(stream_id);
    if (it == s->streams.end() || !it->second.open) return PP_E_INVAL;
    it->second.open = false;
    // queued and admitted-but-not-launched frames are cancelled; launched ones finish
    auto cancel = [&](std::deque<uint64_t>& q) {
        for (auto qi = q.begin(); qi != q.end();) {
            Ticket& t = s->tickets[*qi];
            if (t.stream == stream_id) {
                release_frame(s, t);
                t.state = T_CANCELLED;
                ++s->cancelled;
                qi = q.erase(qi);
            } else {
                ++qi;
            }
        }
    };
    cancel(s->queue);
    cancel(s->ready);
    s->cv_done.notify_all();
    return PP_OK;
}

pp_status pp_submit(pp_server* s, int32_t stream_id, const uint16_t* depth_host, uint64_t frame_id,
                    uint64_t* ticket) {
    if (!s || !depth_host || !ticket) return PP_E_INVAL;
    int slot;
    Stream* st;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->poisoned) return PP_E_HIP;
        auto it = s->streams.find(stream_id);
        if (it == s->streams.end()) return PP_E_INVAL;
        st = &it->second;
        if (!st->open) return PP_E_CLOSED;
        if (st->free_slots.empty()) {
            ++s->rejected;
            return PP_E_AGAIN;  // staging full: the caller retries after polling
        }
        slot = st->free_slots.back();
        st->free_slots.pop_back();
        st->outstanding++;
    }
    // the caller's frame is copied into pinned staging before submit returns
    memcpy(st->in_stage + (size_t)slot * st->in_bytes, depth_host, (size_t)st->desc.width * st->desc.height * 2);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        // a batch may have failed (the scheduler no longer admits anything) or
        // the stream been closed while the frame was copied: the frame is then
        // refused and its slot returned
        if (s->poisoned || !st->open) {
            st->free_slots.push_back(slot);
            st->outstanding--;
            return s->poisoned ? PP_E_HIP : PP_E_CLOSED;
        }
        const uint64_t id = ((uint64_t)(uint32_t)stream_id << 40) | (++s->seq & ((1ull << 40) - 1));
        Ticket t;
        t.stream = stream_id;
        t.frame_id = frame_id;
        t.slot = slot;
        t.t_submit = now_us();
        s->tickets.emplace(id, t);
        s->queue.push_back(id);
        ++s->submitted;
        *ticket = id;
    }
    s->cv_work.notify_all();
    return PP_OK;
}

pp_status pp_poll(pp_server* s, uint64_t ticket, pp_result* out, int32_t timeout_us) {
    if (!s || !out) return PP_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return PP_E_INVAL;
    auto ready = [&] {
        const TicketState st = s->tickets[ticket].state;
        return st == T_DONE || st == T_FAILED || st == T_CANCELLED;
    };
    if (!ready() && timeout_us > 0) s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    Ticket& t = s->tickets[ticket];
    if (!(t.state == T_DONE || t.state == T_FAILED || t.state == T_CANCELLED)) return PP_PENDING;
    Stream& st = s->streams[t.stream];
    pp_status res = PP_OK;
    if (t.state == T_DONE) {
        const char* src = st.out_stage + (size_t)t.slot * st.out_bytes;
        const size_t pb = (size_t)st.rp.max_planes * sizeof(pp_plane);
        if (out->planes) memcpy(out->planes, src, pb);
        if (out->n_planes) memcpy(out->n_planes, src + pb, 4);
        if (out->labels) memcpy(out->labels, src + pb + 256, (size_t)st.desc.width * st.desc.height);
        out->stream_id = t.stream;
        out->frame_id = t.frame_id;
        out->latency_us = t.t_done - t.t_submit;
    } else {
        res = t.state == T_CANCELLED ? PP_E_CLOSED : t.err;
    }
    st.free_slots.push_back(t.slot);
    st.outstanding--;
    s->tickets.erase(ticket);
    return res;
}

pp_status pp_server_reset(pp_server* s) {
    if (!s) return PP_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    // the device work of every lane ends first (a failed batch has ended already)
    if (!s->dry) {
        (void)hipSetDevice(s->cfg.device);
        for (auto& L : s->lanes)
            if (L.stream) (void)hipStreamSynchronize(L.stream);
        (void)hipGetLastError();
    }
    for (auto& L : s->lanes) {
        if (L.busy) {
            if (!s->dry && hipEventQuery(L.done) == hipSuccess) finish_lane(s, L);
            L.busy = false;
            L.dry_fail = false;
            L.tickets.clear();
        }
    }
    // every frame not completed fails; completed results stay pollable
    for (auto& kv : s->tickets) {
        Ticket& t = kv.second;
        if (t.state == T_QUEUED || t.state == T_ADMITTED || t.state == T_INFLIGHT) {
            t.state = T_FAILED;
            t.err = s->poisoned ? PP_E_HIP : PP_E_CLOSED;
        }
        t.bytes = 0;  // the arena is reset below; completed frames released theirs already
    }
    s->queue.clear();
    s->ready.clear();
    const size_t peak = s->arena.peak();
    s->arena.reset(s->cfg.hbm_budget_bytes);
    (void)peak;
    // a context that saw a failure stays poisoned: the lanes get fresh ones
    if (!s->dry) {
        for (auto& L : s->lanes) {
            if (L.ctx) pp_ctx_destroy(L.ctx);
            L.ctx = nullptr;
            if (pp_ctx_create(s->cfg.device, &L.ctx) != PP_OK) {
                L.ctx = nullptr;
                s->poisoned = true;
                s->err = "reset: context re-creation failed";
                s->cv_done.notify_all();
                return PP_E_HIP;
            }
        }
    }
    s->poisoned = false;
    s->err.clear();
    s->cv_done.notify_all();
    s->cv_work.notify_all();
    return PP_OK;
}

pp_status pp_server_stats_get(pp_server* s, pp_server_stats* out) {
    if (!s || !out) return PP_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->rejected = s->rejected;
    out->cancelled = s->cancelled;
    out->launches = s->launches;
    out->mean_batch = s->launches ? (double)s->launched_frames / s->launches : 0.0;
    if (!s->lat.empty()) {
        std::vector<double> v = s->lat;
        auto pct = [&](double q) {
            const size_t k = std::min(v.size() - 1, (size_t)(q * (v.size() - 1) + 0.5));
            std::nth_element(v.begin(), v.begin() + k, v.end());
            return v[k];
        };
        out->p50_us = pct(0.50);
        out->p99_us = pct(0.99);
        out->max_us = *std::max_element(v.begin(), v.end());
    }
    out->hbm_in_use = s->arena.used();
    out->hbm_peak = s->arena.peak();
    out->queued = (int32_t)(s->queue.size() + s->ready.size());
    int inflight = 0;
    for (auto& L : s->lanes) inflight += (int)L.tickets.size();
    out->in_flight = inflight;
    return PP_OK;
}

}  // extern "C"
