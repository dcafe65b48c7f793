// Randomized check of the served form's arena allocator (host-only) against
// a brute-force model: a map of 256-byte units, first fit by linear scan.
// Prints "ok <operations>" on success, "FAIL ..." and exits 1 otherwise.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "fsz_arena.h"

int main(int argc, char **argv)
{
    const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
    const uint64_t units = 4096;  // 1 MiB arena
    fsz::Arena a(units * fsz::Arena::kAlign);
    std::vector<int> owner(units, -1);  // model: allocation id per unit
    std::vector<std::pair<uint64_t, uint64_t>> live;  // (offset, units)
    std::mt19937 rng(seed);
    int ops = 0;
    for (int it = 0; it < 20000; it++) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const uint64_t bytes = (rng() % 3 == 0) ? rng() % 70000 : rng() % 3000;
            const uint64_t need = fsz::Arena::round_up(bytes) / fsz::Arena::kAlign;
            // model first fit
            long long expect = -1;
            uint64_t run = 0;
            for (uint64_t u = 0; u < units; u++) {
                run = owner[u] < 0 ? run + 1 : 0;
                if (run == need) {
                    expect = (long long)(u + 1 - need);
                    break;
                }
            }
            uint64_t off = 0;
            const bool got = a.alloc(bytes, &off);
            if (got != (expect >= 0) || (got && off != (uint64_t)expect * fsz::Arena::kAlign)) {
                std::printf("FAIL alloc %llu bytes: got %d off %llu, model %lld\n", (unsigned long long)bytes,
                            (int)got, (unsigned long long)off, expect);
                return 1;
            }
            if (got) {
                for (uint64_t u = 0; u < need; u++) owner[off / fsz::Arena::kAlign + u] = it;
                live.push_back({off, need});
            }
        } else {
            const size_t k = rng() % live.size();
            const auto e = live[k];
            live.erase(live.begin() + (long)k);
            if (!a.release(e.first)) {
                std::printf("FAIL release %llu\n", (unsigned long long)e.first);
                return 1;
            }
            for (uint64_t u = 0; u < e.second; u++) owner[e.first / fsz::Arena::kAlign + u] = -1;
            if (a.release(e.first)) {
                std::printf("FAIL double release accepted\n");
                return 1;
            }
        }
        uint64_t used = 0;
        for (auto &l : live) used += l.second * fsz::Arena::kAlign;
        if (!a.check() || a.used() != used) {
            std::printf("FAIL invariants after op %d\n", it);
            return 1;
        }
        ops++;
    }
    for (auto &l : live) a.release(l.first);
    if (a.used() != 0 || a.free_ranges() != 1 || !a.check()) {
        std::printf("FAIL not whole again after freeing everything\n");
        return 1;
    }
    std::printf("ok %d\n", ops);
    return 0;
}
