// first_conflict (fsm_spans.h) against brute force over every pair, on random spans that
// touch, nest, repeat and are empty, plus the cases the library's calls produce.
#include <cstdio>
#include <random>
#include <vector>

#include "fsm_spans.h"

using fsm::Span;

static bool conflict(const Span &a, const Span &b)
{
    if (a.end <= a.begin || b.end <= b.begin) return false;
    if (a.read_only && b.read_only) return false;
    return a.begin < b.end && b.begin < a.end;
}

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
    for (int trial = 0; trial < 200000; ++trial) {
        const int n = 1 + (int)(rng() % 7);
        const uintptr_t range = 4 + rng() % 60;
        std::vector<Span> s((size_t)n);
        for (int k = 0; k < n; ++k) {
            const uintptr_t a = rng() % range, len = rng() % 12;
            s[(size_t)k] = {a, rng() % 8 == 0 ? a : a + len, k, rng() % 2 == 0};
        }
        bool want = false;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) want |= conflict(s[(size_t)i], s[(size_t)j]);
        const std::pair<int, int> got = fsm::first_conflict(s);
        CHECK((got.first >= 0) == want);
        if (want) {
            CHECK(got.first != got.second);
            CHECK(conflict(s[(size_t)got.first], s[(size_t)got.second]));
        }
    }
    // maps of a texture batch: in place, shared inputs, an output on another map's input
    const uintptr_t B = 1000;
    CHECK(fsm::first_conflict({{0, B, 0, false}, {B, 2 * B, 1, false}}).first < 0);
    CHECK(fsm::first_conflict({{0, B, 0, true}, {0, B, 1, true}, {B, 2 * B, 0, false}, {2 * B, 3 * B, 1, false}}).first < 0);
    CHECK(fsm::first_conflict({{0, B, 0, true}, {B, 2 * B, 0, false}, {B, 2 * B, 1, true}, {2 * B, 3 * B, 1, false}}).first >= 0);
    CHECK(fsm::first_conflict({{0, B, 0, false}, {B - 8, 2 * B - 8, 1, false}}).first >= 0);
    CHECK(fsm::first_conflict({{0, B, 0, true}, {8, B + 8, 0, false}}).first == 0);
    CHECK(fsm::first_conflict({}).first < 0);
    std::printf("OK\n");
    return 0;
}
