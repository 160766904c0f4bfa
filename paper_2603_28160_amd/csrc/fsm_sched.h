// fsm_sched.h -- the request scheduler of the serving loop: arrivals, admission by device-memory
// footprint, continuous batching over a fixed set of slots.  Host-only C++ with no HIP types:
// the device side is reached through the Executor interface, so the same loop also runs
// against a simulated clock (the dry run).  Not part of the public interface.
#pragma once

#include <cstdint>
#include <map>
#include <vector>

namespace fsm {

// First-fit allocator over the offsets [0, size) of one device arena, 256-byte granules,
// neighbouring free ranges merged on release.
class Arena {
public:
    explicit Arena(int64_t size = 0);
    int64_t size() const { return size_; }
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }
    // offset of a free range of `bytes`, or -1 when none is large enough now
    int64_t alloc(int64_t bytes);
    void release(int64_t offset, int64_t bytes);
    static int64_t round(int64_t bytes) { return (bytes + 255) / 256 * 256; }

private:
    int64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<int64_t, int64_t> free_;   // offset -> length
};

struct SchedConfig {
    int n_slots = 2;          // batches in flight at once (one stream and workspace each)
    int max_batch = 16;       // simulations per batch at most
    int64_t arena_bytes = 0;  // device bytes for the Z-maps the server owns
    bool realtime = true;     // honour arrival times on the wall clock (else all arrive at 0)
};

// One request as the scheduler sees it.
struct SchedRequest {
    double arrival = 0.0;     // seconds after the start of the run
    int64_t zmap_bytes = 0;   // arena bytes it needs while in flight (0: caller-owned Z-map)
};

// Per-request outcome: status (0 = done, negative = a library status code), times in seconds
// after the start, the batch it ran in and the arena offset of its Z-map (-1 if none).
struct SchedResult {
    int status = 1;           // 1 while pending
    double admit = 0.0, start = 0.0, done = 0.0;
    int batch = -1, slot = -1;
    int64_t arena_offset = -1;
};

class Executor {
public:
    virtual ~Executor() = default;
    // seconds since the start of the run
    virtual double now() = 0;
    // Whether the requests `batch` (in order) fit one slot's workspace together.  A batch of
    // one that does not fit is rejected with `status`.
    virtual bool fits(const std::vector<int> &batch, int &status) = 0;
    // Queue the batch on slot `slot` (asynchronously); 0 or a negative status.
    virtual int submit(int slot, const std::vector<int> &batch, const std::vector<SchedResult> &res) = 0;
    // Whether the slot's batch has finished (0/1), or a negative status.
    virtual int poll(int slot) = 0;
    // Nothing to do until `until` (seconds) or until a slot finishes.
    virtual void idle(double until) = 0;
};

// Run every request to completion.  Admission is first come, first served: the oldest
// arrived request takes its arena range as soon as one is free (a request larger than the
// whole arena is rejected with FSM_ENOMEM); a free slot takes the oldest admitted requests,
// up to max_batch of them and as many as fit its workspace, while other slots are still
// running, so later arrivals join the device while earlier batches are in flight.  Returns 0
// or the first executor error.
int run_schedule(const SchedConfig &cfg, const std::vector<SchedRequest> &req, Arena &arena,
                 Executor &ex, std::vector<SchedResult> &out);

}  // namespace fsm
