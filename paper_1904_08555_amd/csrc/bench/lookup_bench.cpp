// Cache-hit latency of sj_specialize from T host threads, through the C ABI
// with no interpreter in the loop (the lookup the paper finds to dominate
// small JIT-specialized calls, ClangJIT section 5.1).
//
// usage: sj_lookup_bench <threads> <calls per thread> [device]
// device >= 0: the key is a runnable LTimes specialization on that HIP device;
// device <  0: the key is compile-only (no GPU is touched).
// Prints one JSON object: per-thread ns per hit (median and maximum).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "sj.h"

int main(int argc, char **argv)
{
    if (argc < 3) {
        std::fprintf(stderr, "usage: %s <threads> <calls per thread> [device]\n", argv[0]);
        return 2;
    }
    const int threads = std::max(1, std::atoi(argv[1]));
    const long calls = std::max(1L, std::atol(argv[2]));
    const int device = argc > 3 ? std::atoi(argv[3]) : 0;
    if (device >= 0 && sj_init(device) != SJ_OK) {
        std::fprintf(stderr, "sj_init: %s\n", sj_last_error());
        return 1;
    }
    sj_spec s{};
    s.struct_size = sizeof s;
    s.dtype = SJ_F64;
    s.layout = SJ_DGZ;
    s.Z = 32768;
    s.G = 32;
    s.D = 96;
    s.NM = 16;
    if (device < 0) s.flags = SJ_FLAG_COMPILE_ONLY;
    sj_handle first = nullptr;
    if (sj_specialize(SJ_LTIMES, &s, &first) != SJ_OK) {   // the miss: compiles once
        std::fprintf(stderr, "sj_specialize: %s\n", sj_last_error());
        return 1;
    }
    std::vector<double> ns(threads, 0.0);
    std::atomic<int> ready{0};
    std::atomic<bool> go{false}, wrong{false};
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&, t] {
            sj_spec mine = s;   // every thread builds its own request for the same key
            sj_handle h = nullptr;
            ready.fetch_add(1);
            while (!go.load(std::memory_order_acquire)) std::this_thread::yield();
            const auto t0 = std::chrono::steady_clock::now();
            for (long i = 0; i < calls; ++i) {
                if (sj_specialize(SJ_LTIMES, &mine, &h) != SJ_OK || h != first) wrong.store(true);
            }
            const auto t1 = std::chrono::steady_clock::now();
            ns[t] = std::chrono::duration<double, std::nano>(t1 - t0).count() / (double)calls;
        });
    while (ready.load() < threads) std::this_thread::yield();
    go.store(true, std::memory_order_release);
    for (auto &th : pool) th.join();
    if (wrong.load()) {
        std::fprintf(stderr, "a hit returned an error or a different handle\n");
        return 1;
    }
    std::vector<double> sorted = ns;
    std::sort(sorted.begin(), sorted.end());
    std::printf("{\"threads\": %d, \"calls_per_thread\": %ld, \"ns_per_hit_median\": %.1f, \"ns_per_hit_max\": %.1f}\n",
                threads, calls, sorted[sorted.size() / 2], sorted.back());
    return 0;
}
