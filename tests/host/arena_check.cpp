// The serving arena (fsm_sched.h) against a granule map: random allocations and releases,
// each allocation at the lowest free run long enough (first fit), -1 exactly when no free
// run is long enough, neighbouring free ranges merged (a full-size allocation succeeds once
// everything is released), and the used and peak byte counts.
#include <cstdio>
#include <random>
#include <vector>

#include "fsm_sched.h"

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);          \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main()
{
    std::mt19937_64 rng(28160);
    for (int trial = 0; trial < 400; ++trial) {
        const int64_t granules = 1 + (int64_t)(rng() % 64);
        const int64_t size = granules * 256 + (int64_t)(rng() % 256);   // a ragged tail is unusable
        fsm::Arena a(size);
        CHECK(a.size() == granules * 256);
        std::vector<char> taken((size_t)granules, 0);
        struct Live { int64_t off, bytes; };
        std::vector<Live> live;
        int64_t used = 0, peak = 0;
        for (int op = 0; op < 300; ++op) {
            if (live.empty() || rng() % 3 != 0) {
                const int64_t bytes = (int64_t)(rng() % (size_t)(granules * 256 / 2 + 2));   // 0 takes one granule
                const int64_t n = (bytes < 1 ? 256 : (bytes + 255) / 256 * 256) / 256;
                int64_t want = -1;   // the lowest start of n free granules
                for (int64_t g = 0; g + n <= granules && want < 0; ++g) {
                    bool ok = true;
                    for (int64_t k = 0; k < n && ok; ++k) ok = !taken[(size_t)(g + k)];
                    if (ok) want = g;
                }
                const int64_t got = a.alloc(bytes);
                CHECK(got == (want < 0 ? -1 : want * 256));
                if (got >= 0) {
                    for (int64_t k = 0; k < n; ++k) taken[(size_t)(want + k)] = 1;
                    live.push_back({got, bytes});
                    used += n * 256;
                    peak = used > peak ? used : peak;
                }
            } else {
                const size_t i = (size_t)(rng() % live.size());
                const Live l = live[i];
                live.erase(live.begin() + (long)i);
                a.release(l.off, l.bytes);
                const int64_t n = (l.bytes < 1 ? 256 : (l.bytes + 255) / 256 * 256) / 256;
                for (int64_t k = 0; k < n; ++k) taken[(size_t)(l.off / 256 + k)] = 0;
                used -= n * 256;
            }
            CHECK(a.used() == used && a.peak() == peak);
        }
        for (const Live &l : live) a.release(l.off, l.bytes);
        CHECK(a.used() == 0);
        CHECK(a.alloc(granules * 256) == 0);   // released ranges merged back into one
    }
    fsm::Arena empty(100);
    CHECK(empty.size() == 0 && empty.alloc(1) == -1);
    std::printf("OK\n");
    return 0;
}
