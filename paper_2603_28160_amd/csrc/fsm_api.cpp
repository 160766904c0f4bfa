// fsm_api.cpp -- the C ABI of libfsm: context, plan, single simulation and roughness.
//
// A call builds the host plan (fsm_plan.cpp), packs it with the device descriptor into one
// pinned staging image, copies that image to the context's device workspace with a single
// stream-ordered transfer, launches fill -> scatter -> roughness on the caller's stream and
// copies the ~100-byte result back.  The Z-map itself never leaves the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "fsm_internal.h"

struct fsm_ctx {
    int device = 0;
    std::string err;
    void *d_ws = nullptr;     // device workspace
    size_t d_bytes = 0;
    void *h_ws = nullptr;     // pinned host staging
    size_t h_bytes = 0;
    fsm_rough *h_out = nullptr;  // pinned result slot
    bool profiling = false;
    hipEvent_t ev[5] = {};       // upload, fill, scatter, rough, end
    fsm_timings timings = {};
    int strategy = fsm::kStrategyBinned;
    int64_t bucket_bytes = (int64_t)2 << 30;
};

namespace {

using fsm::DevSim;
using fsm::Plan;

constexpr int kItersPerItem = 16;   // steps each thread walks per work item and edge point

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int set_err(fsm_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

int hip_err(fsm_ctx *ctx, hipError_t e, const char *where)
{
    std::string m = std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return set_err(ctx, FSM_EDEVICE, m);
}

// Byte layout of one simulation's workspace.  The first `upload` bytes are built on the host
// and copied with one transfer; the rest is device-only scratch.
struct Layout {
    size_t sim, base, tbase, binned, pT, pTf, cs, csf, xc, upload;
    size_t part1, part2, state, out, counts, offsets, cursor, bkey, bidx, total;
    int64_t n_tiles = 0, cap = 0;
};

int64_t tiles_of(int64_t n) { return (n + fsm::kTile - 1) / fsm::kTile; }

Layout layout_of(const Plan &P, int precision, bool binned, int64_t bucket_bytes)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    L.sim = take(sizeof(DevSim));
    L.base = take(sizeof(int64_t));
    L.tbase = take(sizeof(int64_t));
    L.binned = take(sizeof(uint64_t));
    L.pT = take(sizeof(double) * P.pT.size());
    L.pTf = take(sizeof(float) * 4 * (size_t)P.z_n * P.N);
    L.cs = take(sizeof(double) * P.cs.size());
    L.csf = take(sizeof(float) * P.cs.size());
    L.xc = take(sizeof(double) * P.xc.size());
    L.upload = o;
    L.part1 = take(sizeof(fsm::RoughPart1) * fsm::kRoughBlocks);
    L.part2 = take(sizeof(fsm::RoughPart2) * fsm::kRoughBlocks);
    L.state = take(sizeof(fsm::RoughState));
    L.out = take(sizeof(fsm_rough));
    if (binned) {
        L.n_tiles = tiles_of(P.nx) * tiles_of(P.ny);
        const int64_t key_bytes = precision == FSM_F64 ? 8 : 4;
        const int64_t per_item = (int64_t)fsm::kBlock * P.N;
        int64_t cap = bucket_bytes / (key_bytes + 2);
        if (cap > P.n_evals) cap = P.n_evals;
        if (cap < per_item) cap = per_item;             // at least one item per slice
        if (cap > (int64_t)UINT32_MAX) cap = UINT32_MAX; // offsets are 32-bit
        L.cap = cap;
        const int64_t nb = (L.n_tiles + 4095) / 4096;
        L.counts = take(sizeof(uint32_t) * L.n_tiles);
        L.offsets = take(sizeof(uint32_t) * (L.n_tiles + 1));
        L.cursor = take(sizeof(uint32_t) * (L.n_tiles + nb));
        L.bkey = take((size_t)key_bytes * cap);
        L.bidx = take(sizeof(uint16_t) * cap);
    }
    L.total = o;
    return L;
}

int ensure(fsm_ctx *ctx, size_t bytes)
{
    if (ctx->d_bytes < bytes) {
        if (ctx->d_ws) hipFree(ctx->d_ws);
        ctx->d_ws = nullptr;
        ctx->d_bytes = 0;
        hipError_t e = hipMalloc(&ctx->d_ws, bytes);
        if (e != hipSuccess) { ctx->d_ws = nullptr; return hip_err(ctx, e, "hipMalloc(workspace)"); }
        ctx->d_bytes = bytes;
    }
    if (ctx->h_bytes < bytes) {
        if (ctx->h_ws) hipHostFree(ctx->h_ws);
        ctx->h_ws = nullptr;
        ctx->h_bytes = 0;
        hipError_t e = hipHostMalloc(&ctx->h_ws, bytes, hipHostMallocDefault);
        if (e != hipSuccess) { ctx->h_ws = nullptr; return hip_err(ctx, e, "hipHostMalloc(staging)"); }
        ctx->h_bytes = bytes;
    }
    return FSM_OK;
}

void fill_devsim(const Plan &P, const Layout &L, char *dev, void *zmap, DevSim &d)
{
    std::memset(&d, 0, sizeof d);
    d.pT = reinterpret_cast<const double *>(dev + L.pT);
    d.pTf = reinterpret_cast<const float *>(dev + L.pTf);
    d.cs = reinterpret_cast<const double *>(dev + L.cs);
    d.csf = reinterpret_cast<const float *>(dev + L.csf);
    d.xc = reinterpret_cast<const double *>(dev + L.xc);
    d.zmap = zmap;
    d.y_first = P.y_first;
    d.a_e = P.a_e;
    d.x_lo = P.x_lo;
    d.y_lo = P.y_lo;
    d.inv_dd = P.inv_dd;
    d.nx_d = (double)P.nx;
    d.ny_d = (double)P.ny;
    d.nx = P.nx;
    d.ny = P.ny;
    d.tl_c = P.tl_c;
    d.tl_s = P.tl_s;
    d.ts_c = P.ts_c;
    d.ts_s = P.ts_s;
    d.tilt_lead = P.tilt_lead;
    d.tilt_side = P.tilt_side;
    d.z_n = P.z_n;
    d.N = P.N;
    d.S = P.S;
    d.n_steps = (int32_t)P.n_steps;
    d.n_passes = (int32_t)P.n_passes;
    d.ppi = std::min(P.N, fsm::kBlock);
    d.spi = fsm::kBlock / d.ppi;
    d.chunk = d.spi * kItersPerItem;
    d.n_chunks = (int32_t)((P.n_steps + d.chunk - 1) / d.chunk);
    d.n_items = P.n_passes * (int64_t)d.n_chunks * P.z_n;
    d.item_base = 0;
    d.tiles_x = (int32_t)tiles_of(P.nx);
    d.tiles_y = (int32_t)tiles_of(P.ny);
    d.n_sblocks = (int32_t)((P.n_steps + fsm::kBlock - 1) / fsm::kBlock);
    d.n_bitems = P.n_passes * (int64_t)d.n_sblocks * P.z_n;
    d.bitem_base = 0;
    d.tile_base = 0;
}

void fill_image(const Plan &P, const Layout &L, char *host, const DevSim &d)
{
    std::memcpy(host + L.sim, &d, sizeof d);
    const int64_t base0 = 0;
    std::memcpy(host + L.base, &base0, sizeof base0);
    std::memcpy(host + L.tbase, &base0, sizeof base0);
    const uint64_t zero = 0;
    std::memcpy(host + L.binned, &zero, sizeof zero);
    std::memcpy(host + L.pT, P.pT.data(), sizeof(double) * P.pT.size());
    float *pTf = reinterpret_cast<float *>(host + L.pTf);
    for (size_t k = 0; k < (size_t)P.z_n * P.N; ++k) {
        pTf[4 * k] = (float)P.pT[3 * k];
        pTf[4 * k + 1] = (float)P.pT[3 * k + 1];
        pTf[4 * k + 2] = (float)P.pT[3 * k + 2];
        pTf[4 * k + 3] = 0.0f;
    }
    std::memcpy(host + L.cs, P.cs.data(), sizeof(double) * P.cs.size());
    float *csf = reinterpret_cast<float *>(host + L.csf);
    for (size_t k = 0; k < P.cs.size(); ++k) csf[k] = (float)P.cs[k];
    std::memcpy(host + L.xc, P.xc.data(), sizeof(double) * P.xc.size());
}

bool valid_precision(int p) { return p == FSM_F64 || p == FSM_F32; }

void mark(fsm_ctx *ctx, int k, hipStream_t s)
{
    if (ctx->profiling) hipEventRecord(ctx->ev[k], s);
}

// Read the events of a finished call into ctx->timings (phases that did not run read 0).
void collect(fsm_ctx *ctx, bool have_upload, bool have_scatter)
{
    if (!ctx->profiling) return;
    float t[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k) {
        if ((k == 0 && !have_upload) || ((k == 1 || k == 2) && !have_scatter)) continue;
        int a = k, b = k + 1;
        if (hipEventElapsedTime(&t[k], ctx->ev[a], ctx->ev[b]) != hipSuccess) t[k] = 0.0f;
    }
    ctx->timings.upload_ms = t[0];
    ctx->timings.fill_ms = t[1];
    ctx->timings.scatter_ms = t[2];
    ctx->timings.rough_ms = t[3];
    float tot = 0.0f;
    const int first = have_upload ? 0 : 3;
    if (hipEventElapsedTime(&tot, ctx->ev[first], ctx->ev[4]) != hipSuccess) tot = 0.0f;
    ctx->timings.total_ms = tot;
    ctx->timings.valid = 1;
}

}  // namespace

extern "C" {

int fsm_version(void) { return FSM_ABI_VERSION; }

const char *fsm_strerror(int code)
{
    switch (code) {
    case FSM_OK: return "success";
    case FSM_EINVAL: return "invalid argument";
    case FSM_ENOMEM: return "out of memory";
    case FSM_EDEVICE: return "HIP device error";
    case FSM_EAGAIN: return "resources exhausted, try again";
    case FSM_ENOTSUP: return "not supported";
    default: return "unknown status code";
    }
}

int fsm_plan(const fsm_tool *tool, const fsm_cut *cut, const fsm_grid *grid, int precision,
             fsm_plan_info *out)
{
    if (!tool || !cut || !grid || !out || !valid_precision(precision)) return FSM_EINVAL;
    try {
        Plan P;
        std::string err;
        int rc = fsm::build_plan(*tool, *cut, *grid, P, err, false);
        if (rc != FSM_OK) return rc;
        out->r_reach = P.r_reach;
        out->x_start = P.x_start;
        out->y_first = P.y_first;
        out->n_passes = P.n_passes;
        out->n_steps = P.n_steps;
        out->n_evals = P.n_evals;
        out->n_cells = grid->nx * grid->ny;
        out->zmap_bytes = out->n_cells * (precision == FSM_F64 ? 8 : 4);
        P.pT.resize((size_t)P.z_n * P.N * 3);
        P.cs.resize((size_t)P.z_n * P.S * 2);
        P.xc.resize((size_t)P.n_steps);
        out->workspace_bytes = (int64_t)layout_of(P, precision, true, (int64_t)2 << 30).total;
        return FSM_OK;
    } catch (const std::bad_alloc &) {
        return FSM_ENOMEM;
    } catch (...) {
        return FSM_EINVAL;
    }
}

int fsm_edge_points(const fsm_tool *tool, const fsm_cut *cut, double *out)
{
    if (!tool || !cut || !out) return FSM_EINVAL;
    try {
        fsm_grid g{0.0, 0.0, 1.0, 1, 1};
        Plan P;
        std::string err;
        int rc = fsm::build_plan(*tool, *cut, g, P, err, false);
        if (rc != FSM_OK) return rc;
        std::memcpy(out, P.pT.data(), sizeof(double) * P.pT.size());
        return FSM_OK;
    } catch (const std::bad_alloc &) {
        return FSM_ENOMEM;
    } catch (...) {
        return FSM_EINVAL;
    }
}

int fsm_ctx_create(fsm_ctx **out, int device)
{
    if (!out) return FSM_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return FSM_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return FSM_EDEVICE;
    fsm_ctx *c = new (std::nothrow) fsm_ctx;
    if (!c) return FSM_ENOMEM;
    c->device = device;
    if (hipHostMalloc((void **)&c->h_out, sizeof(fsm_rough), hipHostMallocDefault) != hipSuccess) {
        delete c;
        return FSM_ENOMEM;
    }
    *out = c;
    return FSM_OK;
}

int fsm_ctx_set_option(fsm_ctx *ctx, int option, int64_t value)
{
    if (!ctx) return FSM_EINVAL;
    switch (option) {
    case FSM_OPT_ZMAP_STRATEGY:
        if (value != FSM_ZMAP_BINNED && value != FSM_ZMAP_SCATTER)
            return set_err(ctx, FSM_EINVAL, "unknown Z-map strategy");
        ctx->strategy = (int)value;
        return FSM_OK;
    case FSM_OPT_BUCKET_BYTES:
        if (value < ((int64_t)1 << 20)) return set_err(ctx, FSM_EINVAL, "bucket budget below 1 MiB");
        ctx->bucket_bytes = value;
        return FSM_OK;
    default:
        return set_err(ctx, FSM_EINVAL, "unknown option");
    }
}

int fsm_ctx_set_profiling(fsm_ctx *ctx, int on)
{
    if (!ctx) return FSM_EINVAL;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_err(ctx, e, "hipSetDevice");
    if (on && !ctx->ev[0]) {
        for (auto &ev : ctx->ev) {
            e = hipEventCreate(&ev);
            if (e != hipSuccess) return hip_err(ctx, e, "hipEventCreate");
        }
    }
    ctx->profiling = on != 0;
    return FSM_OK;
}

int fsm_last_timings(const fsm_ctx *ctx, fsm_timings *out)
{
    if (!ctx || !out) return FSM_EINVAL;
    *out = ctx->timings;
    return FSM_OK;
}

void fsm_ctx_destroy(fsm_ctx *ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->device);
    for (auto &ev : ctx->ev)
        if (ev) hipEventDestroy(ev);
    if (ctx->d_ws) hipFree(ctx->d_ws);
    if (ctx->h_ws) hipHostFree(ctx->h_ws);
    if (ctx->h_out) hipHostFree(ctx->h_out);
    delete ctx;
}

int fsm_last_error(const fsm_ctx *ctx, char *buf, size_t n)
{
    if (!ctx || !buf || n == 0) return FSM_EINVAL;
    std::snprintf(buf, n, "%s", ctx->err.c_str());
    return FSM_OK;
}

int fsm_simulate(fsm_ctx *ctx, const fsm_tool *tool, const fsm_cut *cut, const fsm_grid *grid,
                 int precision, void *zmap_dev, fsm_rough *out, void *stream)
{
    if (!ctx) return FSM_EINVAL;
    if (!tool || !cut || !grid || !zmap_dev || !valid_precision(precision))
        return set_err(ctx, FSM_EINVAL, "null argument or invalid precision");
    try {
        Plan P;
        std::string err;
        int rc = fsm::build_plan(*tool, *cut, *grid, P, err, true);
        if (rc != FSM_OK) return set_err(ctx, rc, err);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return hip_err(ctx, e, "hipSetDevice");
        const bool binned = ctx->strategy == fsm::kStrategyBinned;
        const Layout L = layout_of(P, precision, binned, ctx->bucket_bytes);
        rc = ensure(ctx, L.total);
        if (rc != FSM_OK) return rc;
        char *dev = static_cast<char *>(ctx->d_ws);
        char *host = static_cast<char *>(ctx->h_ws);
        DevSim d;
        fill_devsim(P, L, dev, zmap_dev, d);
        fill_image(P, L, host, d);
        hipStream_t s = static_cast<hipStream_t>(stream);
        ctx->timings.valid = 0;
        mark(ctx, 0, s);
        e = hipMemcpyAsync(dev, host, L.upload, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(plan)");
        const int64_t n = grid->nx * grid->ny;
        uint64_t *d_binned = reinterpret_cast<uint64_t *>(dev + L.binned);
        const DevSim *d_sim = reinterpret_cast<const DevSim *>(dev + L.sim);
        mark(ctx, 1, s);
        int he;
        if (!binned) {
            he = fsm::launch_fill(zmap_dev, n, precision, stream);
            if (he) return hip_err(ctx, (hipError_t)he, "fill kernel");
        }
        mark(ctx, 2, s);
        if (binned) {
            fsm::BinBuffers bb;
            bb.counts = reinterpret_cast<uint32_t *>(dev + L.counts);
            bb.offsets = reinterpret_cast<uint32_t *>(dev + L.offsets);
            bb.cursor = reinterpret_cast<uint32_t *>(dev + L.cursor);
            bb.bkey = dev + L.bkey;
            bb.bidx = reinterpret_cast<uint16_t *>(dev + L.bidx);
            bb.cap = L.cap;
            const int64_t per_slice = std::max<int64_t>(1, L.cap / ((int64_t)fsm::kBlock * P.N));
            for (int64_t b0 = 0; b0 < d.n_bitems; b0 += per_slice) {
                const int64_t nit = std::min<int64_t>(per_slice, d.n_bitems - b0);
                he = fsm::launch_binned_slice(d_sim, 1, reinterpret_cast<const int64_t *>(dev + L.base),
                                              reinterpret_cast<const int64_t *>(dev + L.tbase), L.n_tiles,
                                              b0, nit, bb, b0 == 0, precision, d_binned, stream);
                if (he) return hip_err(ctx, (hipError_t)he, "binned Z-map kernels");
            }
        } else {
            he = fsm::launch_scatter(d_sim, d, d.n_items, 1, reinterpret_cast<const int64_t *>(dev + L.base),
                                     precision, d_binned, stream);
            if (he) return hip_err(ctx, (hipError_t)he, "scatter kernel");
        }
        mark(ctx, 3, s);
        if (out) {
            he = fsm::launch_rough(zmap_dev, grid->nx, grid->ny, precision, !binned,
                                   reinterpret_cast<fsm::RoughPart1 *>(dev + L.part1),
                                   reinterpret_cast<fsm::RoughPart2 *>(dev + L.part2),
                                   reinterpret_cast<fsm::RoughState *>(dev + L.state),
                                   reinterpret_cast<fsm_rough *>(dev + L.out), d_binned,
                                   P.n_evals, stream);
            if (he) return hip_err(ctx, (hipError_t)he, "roughness kernels");
            e = hipMemcpyAsync(ctx->h_out, dev + L.out, sizeof(fsm_rough), hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(result)");
        } else if (!binned) {
            he = fsm::launch_decode(zmap_dev, n, precision, stream);
            if (he) return hip_err(ctx, (hipError_t)he, "decode kernel");
        }
        mark(ctx, 4, s);
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
        collect(ctx, true, true);
        if (out) *out = *ctx->h_out;
        return FSM_OK;
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

int fsm_roughness(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zmap_dev,
                  fsm_rough *out, void *stream)
{
    if (!ctx) return FSM_EINVAL;
    if (!grid || !zmap_dev || !out || !valid_precision(precision) || grid->nx < 1 || grid->ny < 1 ||
        grid->nx > INT64_MAX / grid->ny)
        return set_err(ctx, FSM_EINVAL, "invalid grid, pointer or precision");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_err(ctx, e, "hipSetDevice");
    Plan P;   // empty tables: only the reduction part of the layout is used
    const Layout L = layout_of(P, precision, false, 0);
    int rc = ensure(ctx, L.total);
    if (rc != FSM_OK) return rc;
    char *dev = static_cast<char *>(ctx->d_ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->timings.valid = 0;
    mark(ctx, 3, s);
    int he = fsm::launch_rough(const_cast<void *>(zmap_dev), grid->nx, grid->ny, precision, false,
                               reinterpret_cast<fsm::RoughPart1 *>(dev + L.part1),
                               reinterpret_cast<fsm::RoughPart2 *>(dev + L.part2),
                               reinterpret_cast<fsm::RoughState *>(dev + L.state),
                               reinterpret_cast<fsm_rough *>(dev + L.out), nullptr, 0, stream);
    if (he) return hip_err(ctx, (hipError_t)he, "roughness kernels");
    e = hipMemcpyAsync(ctx->h_out, dev + L.out, sizeof(fsm_rough), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(result)");
    mark(ctx, 4, s);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
    collect(ctx, false, false);
    *out = *ctx->h_out;
    return FSM_OK;
}

}  // extern "C"
