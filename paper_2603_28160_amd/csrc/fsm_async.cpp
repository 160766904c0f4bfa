// fsm_async.cpp -- asynchronous batches of the C ABI: submit, poll, wait.
//
// A context owns up to FSM_OPT_ASYNC_SLOTS slots, each a non-blocking stream with its own
// workspace, pinned staging and two events.  A submitted batch is planned on the host, packed
// into its slot's staging and queued on the slot's stream (upload, the same launch sequence as
// fsm_simulate_batch, result copy), ordered after the caller's stream by one event and
// ordering later work on the caller's stream after itself by another.  The slot stays taken,
// with the host plans its upload reads, until the batch is waited for; that is also what
// admission counts: a submit finds no free slot, or no room under the HBM budget, and
// returns FSM_EAGAIN without queueing anything.
#include <hip/hip_runtime.h>

#include <new>
#include <string>
#include <vector>

#include "fsm_runtime.h"

using namespace fsm::rt;
using fsm::DevSim;
using fsm::Plan;

namespace fsm {
namespace rt {

void release_async(fsm_ctx *ctx)
{
    for (AsyncSlot &s : ctx->async) {
        if (s.id && s.done) (void)hipEventSynchronize(s.done);
        if (s.start) (void)hipEventDestroy(s.start);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        release(s.ws);
    }
    ctx->async.clear();
}

}  // namespace rt
}  // namespace fsm

namespace {

AsyncSlot *find_batch(fsm_ctx *ctx, uint64_t id)
{
    if (id == 0) return nullptr;
    for (AsyncSlot &s : ctx->async)
        if (s.id == id) return &s;
    return nullptr;
}

// A free slot, created on demand up to the context's limit; nullptr when all are taken.
int free_slot(fsm_ctx *ctx, AsyncSlot *&out)
{
    out = nullptr;
    for (AsyncSlot &s : ctx->async)
        if (!s.id) {
            out = &s;
            return FSM_OK;
        }
    if ((int)ctx->async.size() >= ctx->async_slots) return FSM_OK;
    // slots never move while batches are in flight (at most 16 of them)
    if (ctx->async.capacity() < 16) ctx->async.reserve(16);
    ctx->async.emplace_back();
    AsyncSlot &s = ctx->async.back();
    hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.start, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (s.start) (void)hipEventDestroy(s.start);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        ctx->async.pop_back();
        return hip_err(ctx, e, "slot stream or events");
    }
    out = &s;
    return FSM_OK;
}

}  // namespace

extern "C" {

int fsm_batch_submit(fsm_ctx *ctx, int n, const fsm_job *jobs, int precision, void *stream,
                     uint64_t *batch_id)
{
    if (!ctx) return FSM_EINVAL;
    if (n < 1 || !jobs || !batch_id || !valid_precision(precision))
        return set_err(ctx, FSM_EINVAL, "empty job list, null argument or invalid precision");
    try {
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return hip_err(ctx, e, "hipSetDevice");
        std::vector<Plan> plans((size_t)n);
        std::vector<void *> zmaps((size_t)n);
        for (int k = 0; k < n; ++k) {
            const fsm_job &j = jobs[k];
            if (!j.tool || !j.cut || !j.grid || !j.zmap_dev)
                return set_err(ctx, FSM_EINVAL, "job " + std::to_string(k) + ": null pointer");
            zmaps[k] = j.zmap_dev;
        }
        std::vector<int> rcs((size_t)n, FSM_OK);
        std::vector<std::string> errs((size_t)n);
        fsm::parallel_for(n, [&](int k) {
            rcs[k] = fsm::build_plan(*jobs[k].tool, *jobs[k].cut, *jobs[k].grid, plans[k], errs[k], true);
        });
        for (int k = 0; k < n; ++k)
            if (rcs[k] != FSM_OK) return set_err(ctx, rcs[k], "job " + std::to_string(k) + ": " + errs[k]);
        int rc = check_job_maps(ctx, plans, zmaps, precision);
        if (rc != FSM_OK) return rc;

        AsyncSlot *slot = nullptr;
        rc = free_slot(ctx, slot);
        if (rc != FSM_OK) return rc;
        if (!slot) return set_err(ctx, FSM_EAGAIN, "every asynchronous slot holds a batch not yet waited for");
        std::vector<DevSim> devs;
        const SetLayout L = make_layout(ctx, plans, precision, params_for(ctx, plans, precision), devs);
        if (ctx->hbm_budget > 0 && slot->ws.d_bytes < L.total) {
            size_t held = 0;
            for (const AsyncSlot &s : ctx->async) held += s.ws.d_bytes;
            if (held - slot->ws.d_bytes + L.total > (size_t)ctx->hbm_budget)
                return set_err(ctx, FSM_EAGAIN, "the batch's workspace exceeds the HBM budget");
        }
        rc = ensure(ctx, slot->ws, L.total, L.total - L.sims, (size_t)L.n);
        if (rc != FSM_OK) return rc;
        slot->plans = std::move(plans);
        slot->devs = std::move(devs);
        hipStream_t user = static_cast<hipStream_t>(stream);
        e = hipEventRecord(slot->start, user);
        if (e == hipSuccess) e = hipStreamWaitEvent(slot->stream, slot->start, 0);
        if (e != hipSuccess) return hip_err(ctx, e, "ordering after the caller's stream");
        rc = enqueue_set(ctx, slot->ws, L, slot->plans, slot->devs, zmaps, slot->stream, false);
        if (rc == FSM_OK) {
            e = hipEventRecord(slot->done, slot->stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(user, slot->done, 0);
            if (e != hipSuccess) rc = hip_err(ctx, e, "ordering the caller's stream after the batch");
        }
        if (rc != FSM_OK) {
            // whatever was queued finishes before the slot is reused
            (void)hipStreamSynchronize(slot->stream);
            slot->plans.clear();
            slot->devs.clear();
            return rc;
        }
        slot->id = ctx->next_batch++;
        slot->n = n;
        *batch_id = slot->id;
        return FSM_OK;
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

int fsm_batch_poll(fsm_ctx *ctx, uint64_t batch_id, int *done)
{
    if (!ctx) return FSM_EINVAL;
    if (!done) return set_err(ctx, FSM_EINVAL, "null argument");
    AsyncSlot *s = find_batch(ctx, batch_id);
    if (!s) return set_err(ctx, FSM_EINVAL, "unknown batch");
    const hipError_t e = hipEventQuery(s->done);
    if (e == hipSuccess) {
        *done = 1;
        return FSM_OK;
    }
    if (e == hipErrorNotReady) {
        *done = 0;
        return FSM_OK;
    }
    return hip_err(ctx, e, "hipEventQuery(batch)");
}

int fsm_batch_wait(fsm_ctx *ctx, uint64_t batch_id, fsm_rough *out)
{
    if (!ctx) return FSM_EINVAL;
    AsyncSlot *s = find_batch(ctx, batch_id);
    if (!s) return set_err(ctx, FSM_EINVAL, "unknown batch");
    const hipError_t e = hipEventSynchronize(s->done);
    if (out && e == hipSuccess)
        for (int k = 0; k < s->n; ++k) out[k] = s->ws.h_out[k];
    s->id = 0;
    s->n = 0;
    s->plans.clear();
    s->devs.clear();
    return e == hipSuccess ? FSM_OK : hip_err(ctx, e, "hipEventSynchronize(batch)");
}

}  // extern "C"
