// fsm_serve.cpp -- the serving loop of the C ABI: fsm_serve_run on the device and
// fsm_serve_dry_run against a simulated clock, both driven by the scheduler of fsm_sched.cpp.
//
// Device side: n_slots streams, each with its own workspace (device scratch and image, pinned
// staging, pinned result records) and a completion event.  A batch is planned on the host
// when its slot takes it, uploaded with one copy, run as the batched launch sequence of
// fsm_simulate_batch and its ~100-byte result records copied back; the loop polls the events.
// Server-held Z-maps live in one arena allocation.  Streams keep the default priority.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "fsm_runtime.h"
#include "fsm_sched.h"
#include "fsm_spans.h"

using namespace fsm::rt;
using fsm::parallel_for;
using fsm::DevSim;
using fsm::Plan;

namespace {

constexpr int kMaxSlots = 16;

// The requests that passed validation, with their shape-only plans (no tables).
struct Book {
    std::vector<int> index;            // request number of each valid request
    std::vector<Plan> shape;           // plan without tables, per valid request
    std::vector<fsm::SchedRequest> sched;
};

int check_config(const fsm_serve_config *cfg, int n, const fsm_request *req, const void *out)
{
    if (!cfg || n < 0 || (n > 0 && (!req || !out))) return FSM_EINVAL;
    if (!valid_precision(cfg->precision) || cfg->n_slots < 1 || cfg->n_slots > kMaxSlots ||
        cfg->max_batch < 1 || cfg->arena_bytes < 0 || cfg->slot_bytes <= 0)
        return FSM_EINVAL;
    return FSM_OK;
}

// Validate every request; invalid ones are finished at once with FSM_EINVAL.
Book book_requests(const fsm_serve_config &cfg, int n, const fsm_request *req,
                   fsm_request_result *out)
{
    Book b;
    const int64_t key = cfg.precision == FSM_F64 ? 8 : 4;
    for (int k = 0; k < n; ++k) {
        std::memset(&out[k], 0, sizeof(fsm_request_result));
        out[k].batch = -1;
        out[k].slot = -1;
        const fsm_request &r = req[k];
        Plan P;
        std::string err;
        int rc = (!r.tool || !r.cut || !r.grid || !(r.arrival_s >= 0.0)) ? FSM_EINVAL
                 : fsm::build_plan(*r.tool, *r.cut, *r.grid, P, err, false);
        if (rc != FSM_OK) {
            const double t = cfg.realtime && r.arrival_s >= 0.0 ? r.arrival_s : 0.0;
            out[k].status = rc;
            out[k].admit_s = out[k].start_s = out[k].done_s = t;
            continue;
        }
        fsm::SchedRequest s;
        s.arrival = r.arrival_s;
        s.zmap_bytes = r.zmap_dev ? 0 : P.nx * P.ny * key;
        b.index.push_back(k);
        b.shape.push_back(std::move(P));
        b.sched.push_back(s);
    }
    return b;
}

// Layout of a batch fitted to a slot: the bucket budget shrinks (more slices) until the whole
// image fits slot_bytes; false if even the smallest bucket does not.
bool fit_slot(const fsm_ctx *ctx, const std::vector<Plan> &plans, int precision,
              int64_t slot_bytes, SetLayout &L, std::vector<DevSim> &devs)
{
    return fit_layout(ctx, plans, precision, slot_bytes, params_for(ctx, plans, precision), L, devs);
}

void fill_result(fsm_request_result &o, const fsm::SchedResult &s)
{
    o.status = s.status;
    o.admit_s = s.admit;
    o.start_s = s.start;
    o.done_s = s.done;
    o.batch = s.batch;
    o.slot = s.slot;
}

// ---- device executor ----------------------------------------------------------------------------

class DeviceExecutor final : public fsm::Executor {
public:
    struct Slot {
        Workspace ws;
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        std::vector<int> batch;        // valid-request numbers in flight
    };

    DeviceExecutor(fsm_ctx *ctx, const fsm_serve_config &cfg, const fsm_request *req,
                   const Book &book, fsm_request_result *out)
        : ctx_(ctx), cfg_(cfg), req_(req), book_(book), out_(out), slots_((size_t)cfg.n_slots)
    {
    }
    ~DeviceExecutor() override { teardown(); }

    int setup()
    {
        for (Slot &s : slots_) {
            hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_err(ctx_, e, "hipStreamCreate(slot)");
            e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
            if (e != hipSuccess) return hip_err(ctx_, e, "hipEventCreate(slot)");
            const int rc = ensure(ctx_, s.ws, (size_t)cfg_.slot_bytes, 0, (size_t)cfg_.max_batch);
            if (rc != FSM_OK) return rc == FSM_EDEVICE ? FSM_ENOMEM : rc;
        }
        if (cfg_.arena_bytes > 0) {
            hipError_t e = hipMalloc(&arena_, (size_t)cfg_.arena_bytes);
            if (e != hipSuccess) {
                arena_ = nullptr;
                hip_err(ctx_, e, "hipMalloc(arena)");
                return FSM_ENOMEM;
            }
        }
        t0_ = std::chrono::steady_clock::now();
        return FSM_OK;
    }

    void teardown()
    {
        for (Slot &s : slots_) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            release(s.ws);
            s = Slot();
        }
        if (arena_) (void)hipFree(arena_);
        arena_ = nullptr;
    }

    double now() override
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
    }

    bool fits(const std::vector<int> &batch, int &status) override
    {
        std::vector<Plan> plans;
        for (int v : batch) plans.push_back(book_.shape[v]);
        SetLayout L;
        std::vector<DevSim> devs;
        status = FSM_ENOMEM;
        return fit_slot(ctx_, plans, cfg_.precision, cfg_.slot_bytes, L, devs);
    }

    int submit(int slot, const std::vector<int> &batch, const std::vector<fsm::SchedResult> &res) override
    {
        Slot &s = slots_[slot];
        const int nb = (int)batch.size();
        std::vector<Plan> plans((size_t)nb);
        std::vector<void *> zmaps((size_t)nb);
        std::vector<int> rcs((size_t)nb, FSM_OK);
        std::vector<std::string> errs((size_t)nb);
        parallel_for(nb, [&](int k) {
            const fsm_request &r = req_[book_.index[batch[k]]];
            rcs[k] = fsm::build_plan(*r.tool, *r.cut, *r.grid, plans[k], errs[k], true);
        });
        for (int k = 0; k < nb; ++k) {
            if (rcs[k] != FSM_OK) return set_err(ctx_, rcs[k], errs[k]);
            const fsm_request &r = req_[book_.index[batch[k]]];
            zmaps[k] = r.zmap_dev ? r.zmap_dev
                                  : static_cast<void *>(static_cast<char *>(arena_) + res[batch[k]].arena_offset);
        }
        SetLayout L;
        std::vector<DevSim> devs;
        if (!fit_slot(ctx_, plans, cfg_.precision, cfg_.slot_bytes, L, devs))
            return set_err(ctx_, FSM_ENOMEM, "batch does not fit the slot workspace");
        int rc = ensure(ctx_, s.ws, L.total, L.total - L.sims, (size_t)L.n);
        if (rc != FSM_OK) return rc;
        rc = enqueue_set(ctx_, s.ws, L, plans, devs, zmaps, s.stream, false);
        if (rc != FSM_OK) return rc;
        hipError_t e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) return hip_err(ctx_, e, "hipEventRecord(slot)");
        s.batch = batch;
        return FSM_OK;
    }

    int poll(int slot) override
    {
        Slot &s = slots_[slot];
        const hipError_t e = hipEventQuery(s.done);
        if (e == hipErrorNotReady) return 0;
        if (e != hipSuccess) return hip_err(ctx_, e, "hipEventQuery(slot)");
        for (size_t k = 0; k < s.batch.size(); ++k)
            out_[book_.index[s.batch[k]]].rough = s.ws.h_out[k];
        s.batch.clear();
        return 1;
    }

    void idle(double until) override
    {
        // a short nap keeps the loop's timestamps within tens of microseconds
        const double wait = until - now();
        if (wait > 2e-4) std::this_thread::sleep_for(std::chrono::microseconds(50));
        else std::this_thread::yield();
    }

private:
    fsm_ctx *ctx_;
    const fsm_serve_config &cfg_;
    const fsm_request *req_;
    const Book &book_;
    fsm_request_result *out_;
    std::vector<Slot> slots_;
    void *arena_ = nullptr;
    std::chrono::steady_clock::time_point t0_;
};

// ---- simulated executor ---------------------------------------------------------------------------

class ModelExecutor final : public fsm::Executor {
public:
    ModelExecutor(const fsm_ctx *probe, const fsm_serve_config &cfg, const fsm_serve_model &m,
                  const Book &book)
        : probe_(probe), cfg_(cfg), m_(m), book_(book), busy_until_((size_t)cfg.n_slots, -1.0)
    {
    }
    double now() override { return t_; }
    bool fits(const std::vector<int> &batch, int &status) override
    {
        std::vector<Plan> plans;
        for (int v : batch) plans.push_back(book_.shape[v]);
        SetLayout L;
        std::vector<DevSim> devs;
        status = FSM_ENOMEM;
        return fit_slot(probe_, plans, cfg_.precision, cfg_.slot_bytes, L, devs);
    }
    int submit(int slot, const std::vector<int> &batch, const std::vector<fsm::SchedResult> &) override
    {
        double d = m_.launch_s;
        for (int v : batch) {
            const Plan &P = book_.shape[v];
            d += m_.per_eval_s * (double)P.n_evals + m_.per_cell_s * (double)(P.nx * P.ny);
        }
        busy_until_[slot] = t_ + d;
        return FSM_OK;
    }
    int poll(int slot) override
    {
        if (busy_until_[slot] < 0.0 || t_ < busy_until_[slot]) return 0;
        busy_until_[slot] = -1.0;
        return 1;
    }
    void idle(double until) override
    {
        double next = until;
        for (double b : busy_until_)
            if (b >= 0.0) next = std::min(next, b);
        if (next < 1e300) t_ = std::max(t_, next);
    }

private:
    const fsm_ctx *probe_;
    const fsm_serve_config &cfg_;
    fsm_serve_model m_;
    const Book &book_;
    std::vector<double> busy_until_;
    double t_ = 0.0;
};

}  // namespace

extern "C" {

int fsm_serve_run(fsm_ctx *ctx, const fsm_serve_config *cfg, int n, const fsm_request *req,
                  fsm_request_result *out)
{
    if (!ctx) return FSM_EINVAL;
    if (check_config(cfg, n, req, out) != FSM_OK)
        return set_err(ctx, FSM_EINVAL, "invalid serving configuration or null argument");
    try {
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return hip_err(ctx, e, "hipSetDevice");
        Book book = book_requests(*cfg, n, req, out);
        // requests of one run may share a batch, whose launches write all its maps
        const uintptr_t key = cfg->precision == FSM_F64 ? sizeof(double) : sizeof(float);
        std::vector<fsm::Span> spans;
        for (size_t v = 0; v < book.index.size(); ++v) {
            const uintptr_t b = reinterpret_cast<uintptr_t>(req[book.index[v]].zmap_dev);
            if (b) spans.push_back({b, b + (uintptr_t)book.shape[v].nx * (uintptr_t)book.shape[v].ny * key,
                                    book.index[v], false});
        }
        const std::pair<int, int> o = fsm::first_conflict(std::move(spans));
        if (o.first >= 0)
            return set_err(ctx, FSM_EINVAL, "requests " + std::to_string(std::min(o.first, o.second)) + " and " +
                                                std::to_string(std::max(o.first, o.second)) + ": Z-maps overlap");
        DeviceExecutor ex(ctx, *cfg, req, book, out);
        int rc = ex.setup();
        if (rc != FSM_OK) return rc;
        fsm::SchedConfig sc;
        sc.n_slots = cfg->n_slots;
        sc.max_batch = cfg->max_batch;
        sc.arena_bytes = cfg->arena_bytes;
        sc.realtime = cfg->realtime != 0;
        fsm::Arena arena(cfg->arena_bytes);
        std::vector<fsm::SchedResult> res;
        rc = fsm::run_schedule(sc, book.sched, arena, ex, res);
        ex.teardown();
        if (rc != FSM_OK) return rc;
        for (size_t v = 0; v < book.index.size(); ++v) fill_result(out[book.index[v]], res[v]);
        return FSM_OK;
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

int fsm_serve_dry_run(const fsm_serve_config *cfg, const fsm_serve_model *model, int n,
                      const fsm_request *req, fsm_request_result *out, int64_t *arena_peak)
{
    if (!model || check_config(cfg, n, req, out) != FSM_OK) return FSM_EINVAL;
    if (!(model->launch_s >= 0.0) || !(model->per_eval_s >= 0.0) || !(model->per_cell_s >= 0.0))
        return FSM_EINVAL;
    try {
        fsm_ctx probe;
        Book book = book_requests(*cfg, n, req, out);
        ModelExecutor ex(&probe, *cfg, *model, book);
        fsm::SchedConfig sc;
        sc.n_slots = cfg->n_slots;
        sc.max_batch = cfg->max_batch;
        sc.arena_bytes = cfg->arena_bytes;
        sc.realtime = cfg->realtime != 0;
        fsm::Arena arena(cfg->arena_bytes);
        std::vector<fsm::SchedResult> res;
        const int rc = fsm::run_schedule(sc, book.sched, arena, ex, res);
        if (rc != FSM_OK) return rc;
        for (size_t v = 0; v < book.index.size(); ++v) fill_result(out[book.index[v]], res[v]);
        if (arena_peak) *arena_peak = arena.peak();
        return FSM_OK;
    } catch (const std::bad_alloc &) {
        return FSM_ENOMEM;
    } catch (...) {
        return FSM_EINVAL;
    }
}

}  // extern "C"
