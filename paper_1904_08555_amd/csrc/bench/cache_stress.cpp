// Concurrency check of the specialization cache through the C ABI, without a
// GPU (compile-only keys).  T threads each request, in their own shuffled
// order and several times over, K distinct keys plus one key whose compile
// fails; meanwhile a reader thread polls sj_stats.  Checks: every request for
// a key returns the same handle in every thread, each key compiles exactly
// once, the failing key returns SJ_ERR_COMPILE to every requester and leaves
// no entry.  Built plainly and with ThreadSanitizer on the host code of the
// library and of this program (the data-race check of the cache).
//
// usage: sj_cache_stress <threads> <rounds>; prints one JSON object, exit 0 on success.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "sj.h"

static sj_spec make(int i)
{
    sj_spec s{};
    s.struct_size = sizeof s;
    s.dtype = SJ_F64;
    s.layout = i % 6;
    s.Z = 64 + 8 * i;
    s.G = 3;
    s.D = 12;
    s.NM = 4;
    s.flags = SJ_FLAG_COMPILE_ONLY;
    return s;
}

int main(int argc, char **argv)
{
    const int threads = argc > 1 ? std::max(1, std::atoi(argv[1])) : 8;
    const int rounds = argc > 2 ? std::max(1, std::atoi(argv[2])) : 3;
    constexpr int K = 6;
    sj_stats_t before{};
    before.struct_size = sizeof before;
    if (sj_stats(&before) != SJ_OK) return 1;

    std::vector<std::vector<sj_handle>> got(threads, std::vector<sj_handle>(K, nullptr));
    std::atomic<int> errors{0}, fail_ok{0}, ready{0};
    std::atomic<bool> go{false}, done{false};
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&, t] {
            std::mt19937 rng(1234u + (unsigned)t);
            std::vector<int> order;
            for (int r = 0; r < rounds; ++r)
                for (int i = 0; i <= K; ++i) order.push_back(i);   // i == K: the failing key
            std::shuffle(order.begin(), order.end(), rng);
            ready.fetch_add(1);
            while (!go.load(std::memory_order_acquire)) std::this_thread::yield();
            for (int i : order) {
                sj_spec s = make(i == K ? 0 : i);
                sj_handle h = nullptr;
                if (i == K) {
                    s.flags |= SJ_FLAG_DEBUG_FAIL_COMPILE;
                    if (sj_specialize(SJ_LTIMES, &s, &h) == SJ_ERR_COMPILE && h == nullptr) fail_ok.fetch_add(1);
                    else errors.fetch_add(1);
                    continue;
                }
                if (sj_specialize(SJ_LTIMES, &s, &h) != SJ_OK || h == nullptr) {
                    errors.fetch_add(1);
                    continue;
                }
                if (got[t][i] == nullptr) got[t][i] = h;
                else if (got[t][i] != h) errors.fetch_add(1);
            }
        });
    std::thread reader([&] {
        sj_stats_t st{};
        st.struct_size = sizeof st;
        while (!done.load(std::memory_order_acquire))
            if (sj_stats(&st) != SJ_OK) errors.fetch_add(1);
    });
    while (ready.load() < threads) std::this_thread::yield();
    go.store(true, std::memory_order_release);
    for (auto &th : pool) th.join();
    done.store(true, std::memory_order_release);
    reader.join();

    bool same = true;
    for (int i = 0; i < K; ++i)
        for (int t = 1; t < threads; ++t) same = same && got[t][i] == got[0][i];
    sj_stats_t after{};
    after.struct_size = sizeof after;
    if (sj_stats(&after) != SJ_OK) return 1;
    const unsigned long long compiles = after.compiles - before.compiles;
    const unsigned long long failures = after.compile_failures - before.compile_failures;
    const unsigned long long entries = after.entries - before.entries;
    // every good key compiled once; the failing key compiled at least once and never cached
    const bool ok = errors.load() == 0 && same && fail_ok.load() == threads * rounds && entries == (unsigned)K &&
                    compiles - failures == (unsigned)K && failures >= 1;
    std::printf("{\"threads\": %d, \"rounds\": %d, \"errors\": %d, \"same_handles\": %s, \"compiles\": %llu, "
                "\"compile_failures\": %llu, \"entries\": %llu, \"failed_requests\": %d, \"ok\": %s}\n",
                threads, rounds, errors.load(), same ? "true" : "false", compiles, failures, entries, fail_ok.load(),
                ok ? "true" : "false");
    return ok ? 0 : 1;
}
