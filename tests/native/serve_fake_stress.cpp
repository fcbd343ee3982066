// Host-side stress of the serving scheduler on its fake backend (no GPU),
// built with sanitizers by tests/test_sanitizers.py.
//   single: one thread drives randomized submit / progress / advance / fail /
//           query / release sequences and checks the budget and state rules;
//   threads: submitters, a scheduler thread and a releaser run at once
//           through the C ABI (the server serialises them with its lock).
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "bnormals.h"

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            std::exit(1);                                                    \
        }                                                                    \
    } while (0)

static bn_server *make(int64_t budget, int max_batch, int in_flight) {
    bn_server_config cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    cfg.hbm_budget_bytes = budget;
    cfg.max_batch = max_batch;
    cfg.max_batches_in_flight = in_flight;
    cfg.params.alpha = 2;
    cfg.params.mask_mode = BN_MASK_REL;
    cfg.params.tau = 4.0f;
    cfg.backend = BN_BACKEND_FAKE;
    cfg.fake_ns_per_pixel = 0.5;
    cfg.fake_launch_ns = 3000.0;
    cfg.fake_copy_gbs = 20.0;
    bn_server *s = nullptr;
    CHECK(bn_server_create(&cfg, &s) == BN_OK && s);
    return s;
}

static const float kHostDepth[16] = {1.f};

static uint64_t submit(bn_server *s, std::mt19937_64 &rng) {
    static const int sizes[][2] = {{24, 32}, {48, 64}, {120, 160}, {240, 320}, {7, 5}};
    const auto &hw = sizes[rng() % 5];
    const bool host = rng() % 3 == 0;
    uint64_t id = 0;
    // fake backend: pointers are recorded, never dereferenced
    const float *depth = host ? kHostDepth : reinterpret_cast<const float *>(0x100000);
    const int rc = bn_server_submit(s, depth, host ? 1 : 0, hw[0], hw[1], hw[1], 300.f, 300.f,
                                    hw[1] / 2.f, hw[0] / 2.f, &id);
    CHECK(rc == BN_OK);
    return id;
}

static void single(uint64_t seed) {
    std::mt19937_64 rng(seed);
    const int64_t budget = 8 << 20;
    bn_server *s = make(budget, 1 + (int)(rng() % 8), 1 + (int)(rng() % 3));
    std::vector<uint64_t> live;
    for (int step = 0; step < 4000; ++step) {
        const int op = (int)(rng() % 10);
        if (op < 4) {
            live.push_back(submit(s, rng));
        } else if (op < 6) {
            CHECK(bn_server_progress(s) >= 0);
        } else if (op < 7) {
            CHECK(bn_server_fake_advance(s, 1e-6 * (double)(rng() % 2000)) == BN_OK);
        } else if (op < 8 && !live.empty()) {
            (void)bn_server_fake_fail(s, live[rng() % live.size()]);
        } else if (!live.empty()) {
            const size_t k = rng() % live.size();
            bn_request_info info;
            CHECK(bn_server_query(s, live[k], &info) == BN_OK);
            if (info.state == BN_REQ_DONE || info.state == BN_REQ_FAILED) {
                CHECK(bn_server_release(s, live[k]) == BN_OK);
                live[k] = live.back();
                live.pop_back();
            }
        }
        bn_server_stats st;
        CHECK(bn_server_get_stats(s, &st) == BN_OK);
        CHECK(st.bytes_in_use >= 0 && st.bytes_in_use <= budget);
    }
    bn_server_destroy(s);
}

static void threads(uint64_t seed) {
    bn_server *s = make(16 << 20, 6, 2);
    std::mutex mu;
    std::vector<uint64_t> ids;
    std::atomic<int> submitted{0};
    std::atomic<bool> stop{false};
    const int per = 1500;
    std::vector<std::thread> ts;
    for (int t = 0; t < 3; ++t) {
        ts.emplace_back([&, t] {
            std::mt19937_64 rng(seed + 17 * t);
            for (int k = 0; k < per; ++k) {
                const uint64_t id = submit(s, rng);
                {
                    std::lock_guard<std::mutex> g(mu);
                    ids.push_back(id);
                }
                submitted.fetch_add(1);
            }
        });
    }
    std::thread sched([&] {
        while (!stop.load()) {
            (void)bn_server_progress(s);
            (void)bn_server_fake_advance(s, 5e-4);
        }
    });
    std::thread reaper([&] {
        std::mt19937_64 rng(seed + 99);
        int released = 0;
        while (released < 3 * per) {
            uint64_t id = 0;
            {
                std::lock_guard<std::mutex> g(mu);
                if (!ids.empty()) {
                    const size_t k = rng() % ids.size();
                    id = ids[k];
                    ids[k] = ids.back();
                    ids.pop_back();
                }
            }
            if (!id) continue;
            bn_request_info info;
            CHECK(bn_server_query(s, id, &info) == BN_OK);
            if (info.state == BN_REQ_DONE || info.state == BN_REQ_FAILED) {
                CHECK(bn_server_release(s, id) == BN_OK);
                ++released;
            } else {
                std::lock_guard<std::mutex> g(mu);
                ids.push_back(id);
            }
        }
    });
    for (auto &t : ts) t.join();
    reaper.join();
    stop.store(true);
    sched.join();
    bn_server_stats st;
    CHECK(bn_server_get_stats(s, &st) == BN_OK);
    CHECK(st.completed + st.failed == 3 * per && st.released == 3 * per && st.bytes_in_use == 0);
    bn_server_destroy(s);
}

int main(int argc, char **argv) {
    const char *mode = argc > 1 ? argv[1] : "single";
    if (!std::strcmp(mode, "single")) {
        for (uint64_t seed = 1; seed <= 20; ++seed) single(seed);
    } else {
        threads(7);
    }
    std::printf("ok %s\n", mode);
    return 0;
}
