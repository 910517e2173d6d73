// Driver of the serving runtime's dry-run scheduler for ThreadSanitizer:
// four submitter threads on four streams and one poller thread, a tight
// budget, two lanes, a stream closed while frames are queued, an injected
// batch failure followed by a reset, and stats read concurrently.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <vector>

#include "pp.h"

#define CHECK(x)                                                        \
    do {                                                                \
        if (!(x)) {                                                     \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); \
            std::exit(1);                                               \
        }                                                               \
    } while (0)

int main() {
    const int W = 64, H = 48, kStreams = 4, kFrames = 40;
    pp_server_cfg cfg{};
    cfg.device = 0;
    cfg.hbm_budget_bytes = 8ull << 20;
    cfg.max_batch = 3;
    cfg.lanes = 2;
    cfg.staging_frames = 16;
    cfg.use_graphs = 1;
    cfg.dry_run_us = 300;
    cfg.dry_run_fail_batch = 0;
    pp_server* s = nullptr;
    CHECK(pp_server_create(&cfg, &s) == PP_OK);
    pp_intrinsics K{60.f, 60.f, 32.f, 24.f};
    pp_diffuse_params dp{10, 0.2f, 30.f, PP_EDGE_EXP, PP_DIFFUSE_EDGE4};
    pp_ransac_params rp{12, 128, 50, 0.01f, 1, 0, PP_SCORE_FP32, 0.f};
    for (int i = 0; i < kStreams; ++i) CHECK(pp_stream_open(s, i, pp_frame_desc{W, H, W}, K, &dp, &rp) == PP_OK);
    std::vector<uint16_t> frame((size_t)W * H, 1234);
    std::mutex mu;
    std::vector<uint64_t> pending;
    std::atomic<int> submitted{0}, finished{0}, done_submitting{0};
    auto submitter = [&](int sid) {
        for (int k = 0; k < kFrames; ++k) {
            uint64_t t = 0;
            pp_status st;
            while ((st = pp_submit(s, sid, frame.data(), (uint64_t)k, &t)) == PP_E_AGAIN) std::this_thread::yield();
            if (st == PP_E_CLOSED) break;  // stream 3 is closed midway
            CHECK(st == PP_OK);
            ++submitted;
            std::lock_guard<std::mutex> lk(mu);
            pending.push_back(t);
        }
        ++done_submitting;
    };
    auto poller = [&] {
        std::vector<uint8_t> planes(12 * sizeof(pp_plane));
        int32_t n = 0;
        while (done_submitting.load() < kStreams || finished.load() < submitted.load()) {
            uint64_t t = 0;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (pending.empty()) {
                    t = 0;
                } else {
                    t = pending.front();
                    pending.erase(pending.begin());
                }
            }
            if (!t) {
                std::this_thread::yield();
                continue;
            }
            pp_result r{};
            r.planes = reinterpret_cast<pp_plane*>(planes.data());
            r.n_planes = &n;
            const pp_status st = pp_poll(s, t, &r, 500);
            if (st == PP_PENDING) {
                std::lock_guard<std::mutex> lk(mu);
                pending.push_back(t);
                continue;
            }
            CHECK(st == PP_OK || st == PP_E_CLOSED);
            ++finished;
        }
    };
    auto stats_reader = [&] {
        pp_server_stats st{};
        for (int i = 0; i < 200; ++i) {
            CHECK(pp_server_stats_get(s, &st) == PP_OK);
            std::this_thread::yield();
        }
    };
    std::vector<std::thread> th;
    for (int i = 0; i < kStreams; ++i) th.emplace_back(submitter, i);
    th.emplace_back(poller);
    th.emplace_back(stats_reader);
    std::this_thread::sleep_for(std::chrono::milliseconds(3));
    CHECK(pp_stream_close(s, 3) == PP_OK);
    for (auto& t : th) t.join();
    pp_server_stats st{};
    CHECK(pp_server_stats_get(s, &st) == PP_OK);
    CHECK(st.queued == 0 && st.in_flight == 0 && st.hbm_in_use == 0);
    CHECK(st.completed + st.cancelled == (uint64_t)submitted.load());
    CHECK(pp_server_destroy(s) == PP_OK);

    // an injected failure with a poller waiting, then a reset racing nothing
    cfg.dry_run_fail_batch = 2;
    CHECK(pp_server_create(&cfg, &s) == PP_OK);
    CHECK(pp_stream_open(s, 0, pp_frame_desc{W, H, W}, K, &dp, &rp) == PP_OK);
    std::vector<uint64_t> ts;
    int failed = 0;
    for (int k = 0; k < 8; ++k) {
        uint64_t t = 0;
        // once the injected failure has poisoned the server, submissions are refused
        const pp_status ss = pp_submit(s, 0, frame.data(), (uint64_t)k, &t);
        CHECK(ss == PP_OK || ss == PP_E_HIP);
        if (ss == PP_OK)
            ts.push_back(t);
        else
            ++failed;
    }
    std::thread p2([&] {
        for (uint64_t t : ts) {
            pp_result r{};
            pp_status st;
            while ((st = pp_poll(s, t, &r, 1000)) == PP_PENDING) {
            }
            if (st == PP_E_HIP) ++failed;
        }
    });
    p2.join();
    CHECK(failed > 0);
    CHECK(pp_server_reset(s) == PP_OK);
    uint64_t t = 0;
    CHECK(pp_submit(s, 0, frame.data(), 99, &t) == PP_OK);
    pp_result r{};
    pp_status ps;
    while ((ps = pp_poll(s, t, &r, 1000)) == PP_PENDING) {
    }
    CHECK(ps == PP_OK);
    CHECK(pp_server_destroy(s) == PP_OK);
    std::printf("server_tsan ok: %d submitted, %d finished\n", submitted.load(), finished.load());
    return 0;
}
