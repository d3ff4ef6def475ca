// Stress check of the serving loop's host side, built with AddressSanitizer
// on host code (see build_stress.py).  Three databases are served while six
// threads submit and wait on requests and a seventh keeps pausing and
// resuming databases (the refresh window of Section 4) and reading the
// counters; then the server is drained and every answer is compared bit for
// bit with the oracle's single-query Answer (Definition 1).  Exit 0 and
// "ok ..." on success; a sanitizer report ends the process with the exit
// code set in ASAN_OPTIONS.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "qpir.h"

extern "C" void oracle_answer(const uint8_t* D, uint64_t R, uint64_t C, uint64_t pitch,
                              const uint32_t* q, uint32_t* a);

namespace {

struct Shape {
    uint32_t R, C;
};

struct Req {
    uint32_t db = 0;
    std::vector<uint32_t> q, a;
    uint64_t ticket = 0;
};

int fail(const char* what, pir_status st) {
    std::fprintf(stderr, "FAIL %s: %s\n", what, pir_status_string(st));
    return 1;
}

}  // namespace

int main(int argc, char** argv) {
    const uint32_t graphs = argc > 1 ? (uint32_t)std::atoi(argv[1]) : 1u;
    const Shape shapes[] = {{512, 2048}, {1024, 1024}, {256, 4096}};
    constexpr int kDbs = 3, kThreads = 6, kPer = 120;
    std::mt19937_64 rng(20251003);

    std::vector<std::vector<uint8_t>> hD(kDbs);
    std::vector<uint8_t*> dD(kDbs, nullptr);
    std::vector<pir_db_t*> dbs(kDbs, nullptr);
    int ndev = 0;
    hipError_t he = hipGetDeviceCount(&ndev);
    if (he != hipSuccess || ndev < 1) {
        std::fprintf(stderr, "FAIL hipGetDeviceCount: %s (%d devices)\n", hipGetErrorString(he),
                     ndev);
        return 1;
    }
    for (int d = 0; d < kDbs; ++d) {
        const uint64_t n = (uint64_t)shapes[d].R * shapes[d].C;
        hD[d].resize(n);
        for (auto& x : hD[d]) x = (uint8_t)rng();
        if ((he = hipMalloc(&dD[d], n)) != hipSuccess ||
            (he = hipMemcpy(dD[d], hD[d].data(), n, hipMemcpyHostToDevice)) != hipSuccess) {
            std::fprintf(stderr, "FAIL device buffer: %s\n", hipGetErrorString(he));
            return 1;
        }
        const pir_status st = pir_db_open(dD[d], shapes[d].R, shapes[d].C, shapes[d].C, nullptr,
                                          &dbs[d]);
        if (st != PIR_OK) return fail("pir_db_open", st);
    }

    pir_server_config cfg{};
    cfg.max_batch = 16;
    cfg.slots_per_db = 2;
    cfg.mem_budget_bytes = 64ull << 20;
    cfg.max_queue = 0;
    cfg.use_graphs = graphs;
    cfg.max_inflight = 2;
    pir_server_t* srv = nullptr;
    pir_status st = pir_server_create(&cfg, &srv);
    if (st != PIR_OK) return fail("pir_server_create", st);
    for (int d = 0; d < kDbs; ++d) {
        uint32_t idx = 0;
        if ((st = pir_server_add_db(srv, dbs[d], &idx)) != PIR_OK) return fail("add_db", st);
    }
    if ((st = pir_server_start(srv)) != PIR_OK) return fail("pir_server_start", st);

    // Requests drawn up front, so the submitting threads share no generator.
    std::vector<Req> reqs(kThreads * kPer);
    for (auto& r : reqs) {
        r.db = (uint32_t)(rng() % kDbs);
        r.q.resize(shapes[r.db].C);
        for (auto& w : r.q) w = (uint32_t)rng();
        r.a.assign(shapes[r.db].R, 0u);
    }

    std::atomic<bool> stop{false};
    std::atomic<int> errors{0};
    std::thread admin([&] {
        std::mt19937 g(7);
        while (!stop.load()) {
            const uint32_t d = g() % kDbs;
            if (pir_server_pause_db(srv, d) != PIR_OK) ++errors;
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            if (pir_server_resume_db(srv, d) != PIR_OK) ++errors;
            pir_server_stats s{};
            if (pir_server_stats_get(srv, &s) != PIR_OK) ++errors;
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
    });
    std::vector<std::thread> subs;
    for (int t = 0; t < kThreads; ++t) {
        subs.emplace_back([&, t] {
            for (int i = 0; i < kPer; ++i) {
                Req& r = reqs[t * kPer + i];
                if (pir_server_submit(srv, r.db, r.q.data(), r.a.data(), 0, &r.ticket) != PIR_OK)
                    ++errors;
                // Wait on an earlier request now and then, as a client would.
                if (i % 8 == 7 &&
                    pir_server_wait(srv, reqs[t * kPer + i - 3].ticket, UINT64_MAX) != PIR_OK)
                    ++errors;
            }
        });
    }
    for (auto& th : subs) th.join();
    stop = true;
    admin.join();
    if ((st = pir_server_drain(srv)) != PIR_OK) return fail("pir_server_drain", st);
    if (errors.load()) {
        std::fprintf(stderr, "FAIL %d calls returned an error\n", errors.load());
        return 1;
    }

    pir_server_stats s{};
    if ((st = pir_server_stats_get(srv, &s)) != PIR_OK) return fail("stats", st);
    if (s.completed != reqs.size() || s.failed != 0) {
        std::fprintf(stderr, "FAIL completed %llu failed %llu of %zu\n",
                     (unsigned long long)s.completed, (unsigned long long)s.failed, reqs.size());
        return 1;
    }
    if ((st = pir_server_destroy(srv)) != PIR_OK) return fail("pir_server_destroy", st);

    int bad = 0;
    std::vector<uint32_t> want;
    for (const Req& r : reqs) {
        const Shape sh = shapes[r.db];
        want.assign(sh.R, 0u);
        oracle_answer(hD[r.db].data(), sh.R, sh.C, sh.C, r.q.data(), want.data());
        if (want != r.a) ++bad;
    }
    for (int d = 0; d < kDbs; ++d) {
        pir_db_close(dbs[d]);
        (void)hipFree(dD[d]);
    }
    if (bad) {
        std::fprintf(stderr, "FAIL %d of %zu answers differ from the oracle\n", bad, reqs.size());
        return 1;
    }
    std::printf("ok: %zu requests over %d databases, graphs=%u, %llu batches\n", reqs.size(),
                kDbs, graphs, (unsigned long long)s.batches);
    return 0;
}
