// Host check of the planner's thread pool (parallel_for over pool_run): every index runs
// exactly once, nested loops run inline, several host threads may call at once, the first
// exception reaches the caller, and a forked child runs its loops inline.
#include <atomic>
#include <cstdio>
#include <stdexcept>
#include <sys/wait.h>
#include <thread>
#include <unistd.h>
#include <vector>

#include "fsm_internal.h"

static int fail(const char *what)
{
    std::printf("FAIL %s\n", what);
    return 1;
}

int main()
{
    // every index once
    for (int n : {0, 1, 2, 3, 17, 1000, 100000}) {
        std::vector<std::atomic<int>> hits((size_t)n);
        for (auto &h : hits) h = 0;
        fsm::parallel_for(n, [&](int k) { hits[(size_t)k]++; });
        for (auto &h : hits)
            if (h != 1) return fail("coverage");
    }
    // nested loops
    std::atomic<long> total{0};
    fsm::parallel_for(64, [&](int) { fsm::parallel_for(100, [&](int k) { total += k; }); });
    if (total != 64L * 4950) return fail("nested");
    // concurrent callers
    std::atomic<long> sum{0};
    std::vector<std::thread> ts;
    for (int t = 0; t < 6; ++t)
        ts.emplace_back([&] {
            for (int r = 0; r < 50; ++r) fsm::parallel_for(257, [&](int k) { sum += k; });
        });
    for (auto &t : ts) t.join();
    if (sum != 6L * 50 * (256L * 257 / 2)) return fail("concurrent");
    // exceptions
    bool caught = false;
    try {
        fsm::parallel_for(500, [&](int k) {
            if (k == 321) throw std::runtime_error("planted");
        });
    } catch (const std::runtime_error &) {
        caught = true;
    }
    if (!caught) return fail("exception");
    std::atomic<int> after{0};
    fsm::parallel_for(100, [&](int) { after++; });
    if (after != 100) return fail("after exception");
    // a forked child does not own the pool's threads: its loops run inline and finish
    const pid_t pid = fork();
    if (pid == 0) {
        std::atomic<int> c{0};
        fsm::parallel_for(1000, [&](int) { c++; });
        _exit(c == 1000 ? 0 : 3);
    }
    int st = 0;
    waitpid(pid, &st, 0);
    if (!WIFEXITED(st) || WEXITSTATUS(st) != 0) return fail("fork");
    std::printf("OK\n");
    return 0;
}
