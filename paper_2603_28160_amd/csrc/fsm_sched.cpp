// fsm_sched.cpp -- the serving loop's scheduler (host only; see fsm_sched.h).
#include "fsm_sched.h"

#include <algorithm>
#include <deque>
#include <numeric>

#include "../../include/fsm.h"

namespace fsm {

Arena::Arena(int64_t size) : size_(size / 256 * 256)
{
    if (size_ > 0) free_[0] = size_;
}

int64_t Arena::alloc(int64_t bytes)
{
    const int64_t n = round(bytes < 1 ? 1 : bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < n) continue;
        const int64_t at = it->first, left = it->second - n;
        free_.erase(it);
        if (left > 0) free_[at + n] = left;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return at;
    }
    return -1;
}

void Arena::release(int64_t offset, int64_t bytes)
{
    const int64_t n = round(bytes < 1 ? 1 : bytes);
    used_ -= n;
    auto next = free_.lower_bound(offset);
    int64_t at = offset, len = n;
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == at) {
            at = prev->first;
            len += prev->second;
            free_.erase(prev);
        }
    }
    if (next != free_.end() && at + len == next->first) {
        len += next->second;
        free_.erase(next);
    }
    free_[at] = len;
}

int run_schedule(const SchedConfig &cfg, const std::vector<SchedRequest> &req, Arena &arena,
                 Executor &ex, std::vector<SchedResult> &out)
{
    const int n = (int)req.size();
    out.assign((size_t)n, SchedResult());
    // arrival order (stable: equal times keep the caller's order)
    std::vector<int> order((size_t)n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return req[a].arrival < req[b].arrival; });
    size_t next_arrival = 0;
    std::deque<int> waiting;     // arrived, not yet admitted
    std::deque<int> admitted;    // holding their arena range, not yet started
    std::vector<std::vector<int>> running((size_t)cfg.n_slots);
    int finished = 0, batches = 0;

    auto arrival_time = [&](int r) { return cfg.realtime ? req[r].arrival : 0.0; };
    auto finish = [&](int r, int status, double t) {
        SchedResult &o = out[r];
        o.status = status;
        o.done = t;
        if (o.arena_offset >= 0) arena.release(o.arena_offset, req[r].zmap_bytes);
        ++finished;
    };

    while (finished < n) {
        double t = ex.now();
        // 1. completions free slots and arena ranges
        for (int s = 0; s < cfg.n_slots; ++s) {
            if (running[s].empty()) continue;
            const int p = ex.poll(s);
            if (p < 0) return p;
            if (p == 1) {
                t = ex.now();
                for (int r : running[s]) finish(r, 0, t);
                running[s].clear();
            }
        }
        // 2. arrivals
        while (next_arrival < order.size() && arrival_time(order[next_arrival]) <= t)
            waiting.push_back(order[next_arrival++]);
        // 3. admission, oldest first: stop at the first request that must wait for memory
        while (!waiting.empty()) {
            const int r = waiting.front();
            if (req[r].zmap_bytes > 0) {
                if (Arena::round(req[r].zmap_bytes) > arena.size()) {
                    waiting.pop_front();
                    out[r].admit = t;
                    finish(r, FSM_ENOMEM, t);
                    continue;
                }
                const int64_t at = arena.alloc(req[r].zmap_bytes);
                if (at < 0) break;
                out[r].arena_offset = at;
            }
            out[r].admit = t;
            admitted.push_back(r);
            waiting.pop_front();
        }
        // 4. free slots take the oldest admitted requests
        for (int s = 0; s < cfg.n_slots && !admitted.empty(); ++s) {
            if (!running[s].empty()) continue;
            std::vector<int> batch;
            while (!admitted.empty() && (int)batch.size() < cfg.max_batch) {
                batch.push_back(admitted.front());
                int status = 0;
                if (!ex.fits(batch, status)) {
                    batch.pop_back();
                    if (batch.empty()) {
                        // alone it does not fit a slot: reject it
                        const int r = admitted.front();
                        admitted.pop_front();
                        finish(r, status ? status : FSM_ENOMEM, t);
                        continue;
                    }
                    break;
                }
                admitted.pop_front();
            }
            if (batch.empty()) continue;
            t = ex.now();
            for (int r : batch) {
                out[r].start = t;
                out[r].batch = batches;
                out[r].slot = s;
            }
            const int rc = ex.submit(s, batch, out);
            if (rc < 0) return rc;
            running[s] = batch;
            ++batches;
        }
        if (finished >= n) break;
        // 5. wait for the next event: an arrival or a completion
        bool busy = false;
        for (auto &b : running) busy = busy || !b.empty();
        const double next_t = next_arrival < order.size() ? arrival_time(order[next_arrival]) : 1e300;
        if (!busy && admitted.empty() && waiting.empty() && next_t >= 1e300) break;   // defensive
        const bool can_start = !admitted.empty() &&
                               std::any_of(running.begin(), running.end(),
                                           [](const std::vector<int> &b) { return b.empty(); });
        if (!can_start) ex.idle(next_t);
    }
    return 0;
}

}  // namespace fsm
