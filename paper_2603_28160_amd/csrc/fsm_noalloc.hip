// fsm_noalloc.hip -- fsm_simulate_noalloc: one simulation without any device or pinned-host
// allocation, for callers that cannot allocate (work under HIP graph capture, tight serving
// loops, harnesses that forbid it).
//
// Its scratch -- roughness partials, counters, the row matrix and buckets of the binned Z-map,
// and the uploaded plan image -- is `scratch`, a fixed device array of this file.  Each GPU the
// library runs on holds its own copy until the process ends.  In host code the array's name
// stands for a host-side shadow, not a device address: the device address is looked up once
// per device with hipGetSymbolAddress (fsm_ctx_create calls noalloc_setup with the device
// current) and only that address is ever passed to a copy or a kernel.  The work runs as the
// launch sequence of fsm_simulate, with the bucket budget cut so the whole workspace fits the
// array (more slices of the binned Z-map where it must).  Every call on a GPU shares the array
// and rewrites everything it reads: the counters and the image travel with each call's upload,
// and the kernels clear their counts themselves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fsm_runtime.h"

namespace {

constexpr size_t kScratchBytes = FSM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct ScratchTable {
    std::mutex m;
    bool looked_up[kMaxDevices] = {};
    hipError_t status[kMaxDevices] = {};
    void *ptr[kMaxDevices] = {};
};

ScratchTable &table()
{
    static ScratchTable *t = new ScratchTable;   // never destroyed: calls may outlive statics
    return *t;
}

}  // namespace

namespace fsm {
namespace rt {

int noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return FSM_EDEVICE;
    ScratchTable &t = table();
    std::lock_guard<std::mutex> g(t.m);
    if (!t.looked_up[device]) {
        void *p = nullptr;
        t.status[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        t.ptr[device] = t.status[device] == hipSuccess ? p : nullptr;
        t.looked_up[device] = true;
    }
    return t.status[device] == hipSuccess ? FSM_OK : FSM_EDEVICE;
}

namespace {

// The device address of the scratch on `device`, or nullptr with the lookup's error.
void *scratch_ptr(int device, hipError_t &e)
{
    ScratchTable &t = table();
    std::lock_guard<std::mutex> g(t.m);
    if (device < 0 || device >= kMaxDevices || !t.looked_up[device]) {
        e = hipErrorInvalidDevice;
        return nullptr;
    }
    e = t.status[device];
    return t.ptr[device];
}

}  // namespace
}  // namespace rt
}  // namespace fsm

extern "C" int fsm_simulate_noalloc(fsm_ctx *ctx, const fsm_tool *tool, const fsm_cut *cut,
                                    const fsm_grid *grid, int precision, void *zmap_dev,
                                    fsm_rough *out, void *stream)
{
    using namespace fsm::rt;
    if (!ctx) return FSM_EINVAL;
    if (!tool || !cut || !grid || !zmap_dev || !valid_precision(precision))
        return set_err(ctx, FSM_EINVAL, "null argument or invalid precision");
    try {
        std::vector<fsm::Plan> plans(1);
        std::string err;
        int rc = fsm::build_plan(*tool, *cut, *grid, plans[0], err, true);
        if (rc != FSM_OK) return set_err(ctx, rc, err);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return hip_err(ctx, e, "hipSetDevice");
        void *base = scratch_ptr(ctx->device, e);
        if (!base) return hip_err(ctx, e, "hipGetSymbolAddress(scratch)");
        // the context's launch parameters, with the row matrix and the buckets cut to the
        // array (the row matrix to a quarter of it; the buckets to what is left)
        LaunchParams lp = params_for(ctx, plans, precision);
        lp.hist_bytes = std::min<int64_t>(lp.hist_bytes, (int64_t)kScratchBytes / 4);
        SetLayout L;
        std::vector<fsm::DevSim> devs;
        if (!fit_layout(ctx, plans, precision, (int64_t)kScratchBytes, lp, L, devs))
            return set_err(ctx, FSM_EINVAL, "simulation needs more than the " +
                                                std::to_string(kScratchBytes >> 20) +
                                                " MiB fixed scratch of fsm_simulate_noalloc");
        // pageable host staging for the plan image and the result record: the copies stage
        // through the runtime's own buffers
        std::vector<char> image(L.total - L.sims);
        fsm_rough rec;
        Workspace w;
        w.d_ws = base;
        w.d_bytes = kScratchBytes;
        w.h_ws = image.data();
        w.h_bytes = image.size();
        w.h_out = &rec;
        w.h_out_n = 1;
        std::vector<void *> zmaps{zmap_dev};
        hipStream_t s = static_cast<hipStream_t>(stream);
        ctx->timings.valid = 0;
        rc = enqueue_set(ctx, w, L, plans, devs, zmaps, s, false);
        if (rc != FSM_OK) return rc;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
        if (out) std::memcpy(out, &rec, sizeof rec);
        return FSM_OK;
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}
