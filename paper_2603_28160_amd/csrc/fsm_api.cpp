// fsm_api.cpp -- the C ABI of libfsm: context, plan, simulations (one or a batch), roughness.
//
// A call builds the host plan of every simulation (fsm_plan.cpp), packs the device
// descriptors and tables into one pinned staging image, copies it to the context's device
// workspace with a single stream-ordered transfer, launches the Z-map strategy and the tiled
// roughness over the whole set at once, and copies the ~100-byte result records back.  The
// Z-maps themselves never leave the device.
//
// Workspace layout: device-only scratch first (its offsets depend only on the launch shape, so
// a captured graph stays valid for every set of that shape), then the uploaded image.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "fsm_runtime.h"
#include "fsm_spans.h"

namespace fsm {
namespace rt {

constexpr int kItersPerItem = 16;   // steps each thread walks per scatter item and edge point

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

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Bytes of bucket space per point: key and cell index, and with super-tiles the super-tile
// bucket's key and 32-bit cell besides.
int64_t entry_bytes(int precision, bool super)
{
    const int64_t key_bytes = precision == FSM_F64 ? 8 : 4;
    return key_bytes + 2 + (super ? key_bytes + 4 : 0);
}

// Bucket capacity in points: the bucket budget over the bytes of one entry, at least one
// binning item's worst case and at most what 32-bit offsets address.
int64_t bucket_cap(int64_t bucket_bytes, int64_t entry, int64_t per_item)
{
    int64_t cap = bucket_bytes / entry;
    cap = std::max<int64_t>(cap, per_item);
    return std::min<int64_t>(cap, (int64_t)UINT32_MAX);
}

bool valid_tile_shape(const fsm_ctx *ctx, int precision, int code)
{
    const int sx = code >> 4, sy = code & 15;
    const size_t key = precision == FSM_F64 ? 8 : 4;
    // the tile's keys live in LDS during the reduction; cell indices inside a tile are 16-bit
    return code >= 0 && (code >> 8) == 0 && sx >= 4 && sx <= 8 && sy >= 4 && sy <= 8 &&
           (key << (sx + sy)) <= ctx->max_lds;
}

void choose_tiles(const fsm_ctx *ctx, int precision, int code, int &sx, int &sy)
{
    if (code != 0 && valid_tile_shape(ctx, precision, code)) {
        sx = code >> 4;
        sy = code & 15;
        return;
    }
    sx = fsm::tile_sx(precision);
    sy = fsm::tile_sy(precision);
    const size_t key = precision == FSM_F64 ? 8 : 4;
    // leave room for the kernel's own small shared arrays
    while (sy > 4 && (key << (sx + sy)) + 1024 > ctx->max_lds) --sy;
}

// binary order of magnitude, for the workload class
int order2(double v) { return v < 1.0 ? 0 : (int)std::floor(std::log2(v) + 0.5); }

std::string tune_key(const std::vector<Plan> &plans, int precision)
{
    double cells = 0.0, evals = 0.0;
    for (const Plan &P : plans) {
        cells += (double)P.nx * (double)P.ny;
        evals += (double)P.n_evals;
    }
    return std::to_string(precision) + "/" + std::to_string(order2((double)plans.size())) + "/" +
           std::to_string(order2(cells)) + "/" + std::to_string(order2(evals));
}

LaunchParams params_for(const fsm_ctx *ctx, const std::vector<Plan> &plans, int precision)
{
    LaunchParams lp;
    lp.strategy = ctx->strategy;
    lp.tile_shape = ctx->tile_shape;
    lp.target_rows = ctx->target_rows;
    lp.bucket_bytes = ctx->bucket_bytes;
    lp.hist_bytes = ctx->hist_bytes;
    if (ctx->use_tuned && !ctx->tuned.empty()) {
        auto it = ctx->tuned.find(tune_key(plans, precision));
        if (it != ctx->tuned.end()) {
            lp.strategy = it->second.strategy;
            lp.tile_shape = it->second.tile_shape;
            lp.target_rows = it->second.target_rows;
        }
    }
    return lp;
}

SetLayout make_layout(const fsm_ctx *ctx, const std::vector<Plan> &plans, int precision,
                      const LaunchParams &lp, std::vector<DevSim> &devs)
{
    const int strategy = lp.strategy;
    const int64_t bucket_bytes = lp.bucket_bytes;
    SetLayout L;
    L.n = (int)plans.size();
    L.precision = precision;
    L.strategy = strategy;
    choose_tiles(ctx, precision, lp.tile_shape, L.sx, L.sy);
    devs.assign(L.n, DevSim{});
    int64_t items = 0, bitems = 0, tiles = 0, groups = 0;
    for (int k = 0; k < L.n; ++k) {
        const Plan &P = plans[k];
        DevSim &d = devs[k];
        std::memset(&d, 0, sizeof d);
        d.y_first = P.y_first;
        d.a_e = P.a_e;
        d.x_start = P.x_start;
        d.feed = P.feed;
        d.dt = P.dt;
        d.fixed_dt = P.fixed_dt ? 1 : 0;
        d.x_lo = P.x_lo;
        d.y_lo = P.y_lo;
        d.inv_dd = P.inv_dd;
        d.nx_d = (double)P.nx;
        d.ny_d = (double)P.ny;
        d.nx = P.nx;
        d.ny = P.ny;
        d.n_groups = P.n_groups;
        d.x_hi = P.x_hi;
        d.y_hi = P.y_hi;
        d.cull_reach = P.cull_reach;
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
        d.ppi = std::max(1, std::min(P.N, fsm::kBlock));
        d.spi = fsm::kBlock / d.ppi;
        d.chunk = d.spi * kItersPerItem;
        d.n_chunks = (int32_t)ceil_div(P.n_steps, d.chunk);
        d.n_items = P.n_passes * (int64_t)d.n_chunks * P.z_n;
        d.item_base = items;
        items += d.n_items;
        d.n_sblocks = (int32_t)ceil_div(P.n_steps, fsm::kBlock);
        d.n_bitems = P.n_passes * (int64_t)d.n_sblocks * P.z_n;
        d.bitem_base = bitems;
        bitems += d.n_bitems;
        d.sx = L.sx;
        d.sy = L.sy;
        d.tiles_x = (int32_t)ceil_div(P.nx, (int64_t)1 << L.sx);
        d.tiles_y = (int32_t)ceil_div(P.ny, (int64_t)1 << L.sy);
        d.n_tiles = (int64_t)d.tiles_x * d.tiles_y;
        d.tile_base = tiles;
        tiles += d.n_tiles;
        d.ux = d.uy = 0;
        d.h_tiles_x = d.tiles_x;
        d.h_tiles = d.n_tiles;
        d.h_base = d.tile_base;
        // reduction groups of the binned strategy: the largest power of two of tiles (up to
        // 64) that still leaves kReduceGroups groups; it follows from the simulation's own
        // tiles only, so a simulation reduces alike alone and in a batch.  The scatter
        // strategy's first pass (and the roughness of given maps) leaves a partial per tile.
        d.tg_shift = 0;
        while (strategy == fsm::kStrategyBinned && d.tg_shift < fsm::kMaxGroupShift &&
               (d.n_tiles >> (d.tg_shift + 1)) >= fsm::kReduceGroups)
            ++d.tg_shift;
        d.n_tgroups = ceil_div(d.n_tiles, (int64_t)1 << d.tg_shift);
        d.tgroup_base = groups;
        groups += d.n_tgroups;
        d.sim = k;
        if (precision == FSM_F32) {
            d.pos_err = fsm::kF32PosErr * P.pos_r;
            d.near_w = d.pos_err * P.inv_dd * (1.0 + 0x1p-20) + 0x1p-30;
        } else {
            d.pos_err = 0.0;
            d.near_w = -1.0;
        }
        L.max_n = std::max(L.max_n, P.N);
    }
    L.total_tiles = tiles;
    L.total_htiles = tiles;
    L.total_groups = groups;
    const bool binned = strategy == fsm::kStrategyBinned;
    L.total_items = binned ? bitems : items;
    if (binned) {
        // histogram mode when every simulation's row histogram fits in LDS and the row matrix
        // fits its budget; simulations with more tiles than a histogram holds count per
        // super-tile, grown along its shorter side (in cells) until a histogram holds at most
        // kSuperHistTiles of them.
        int64_t max_tiles = 0;
        for (const DevSim &d : devs) max_tiles = std::max(max_tiles, d.n_tiles);
        int ux = 0, uy = 0;
        int64_t max_h = max_tiles;
        if (max_tiles > fsm::kMaxHistTiles) {
            for (;;) {
                max_h = 0;
                for (const DevSim &d : devs)
                    max_h = std::max(max_h, ceil_div(d.tiles_x, (int64_t)1 << ux) * ceil_div(d.tiles_y, (int64_t)1 << uy));
                if (max_h <= fsm::kSuperHistTiles || ux + uy >= fsm::kMaxSubShift) break;
                if (L.sx + ux <= L.sy + uy) ++ux; else ++uy;
            }
            if (max_h > fsm::kMaxHistTiles) ux = uy = 0;
        }
        const bool super = ux + uy > 0;
        if (super) {
            int64_t htiles = 0;
            for (DevSim &d : devs) {
                d.ux = ux;
                d.uy = uy;
                d.h_tiles_x = (int32_t)ceil_div(d.tiles_x, (int64_t)1 << ux);
                d.h_tiles = d.h_tiles_x * ceil_div(d.tiles_y, (int64_t)1 << uy);
                d.h_base = htiles;
                htiles += d.h_tiles;
            }
            L.total_htiles = htiles;
        }
        L.entry = entry_bytes(precision, super);
        // Rows: about target_rows per launch, that is per slice when the work runs in several
        // (a row never holds more items than one bucket slice can take); coarser only when the
        // row matrix would outgrow its budget.
        const int64_t per_item = (int64_t)fsm::kBlock * L.max_n;
        const int64_t slice_items = std::max<int64_t>(
            1, std::min(bucket_cap(bucket_bytes, L.entry, per_item), std::max(per_item, bitems * per_item)) / per_item);
        int64_t ipr = std::max<int64_t>(1, ceil_div(std::min(bitems, slice_items), std::max<int64_t>(1, lp.target_rows)));
        int64_t rows = 0, hsize = 0;
        for (;;) {
            rows = hsize = 0;
            for (DevSim &d : devs) {
                d.items_per_row = (int32_t)ipr;
                d.n_rows = ceil_div(d.n_bitems, ipr);
                d.row_base = rows;
                d.hbase = hsize;
                rows += d.n_rows;
                hsize += d.n_rows * d.h_tiles;
            }
            if (hsize * 4 <= lp.hist_bytes || ipr >= slice_items) break;
            ipr = std::min(slice_items, ipr * 2);
        }
        L.items_per_row = ipr;
        L.total_rows = rows;
        L.max_tiles = 0;
        for (const DevSim &d : devs) L.max_tiles = std::max(L.max_tiles, d.h_tiles);
        L.hist = L.max_tiles <= fsm::kMaxHistTiles && hsize * 4 <= lp.hist_bytes;
        L.super = L.hist && super;
        if (!L.hist) {
            // run mode: global atomics per tile
            L.max_tiles = 0;
            L.total_htiles = tiles;
            L.entry = entry_bytes(precision, false);
            for (DevSim &d : devs) {
                d.ux = d.uy = 0;
                d.h_tiles_x = d.tiles_x;
                d.h_tiles = d.n_tiles;
                d.h_base = d.tile_base;
            }
        }
    }

    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    L.st1 = take(sizeof(fsm::TileStat1) * tiles);
    L.st2 = take(sizeof(fsm::TileStat2) * tiles);
    L.state = take(sizeof(fsm::RoughState) * L.n);
    L.out = take(sizeof(fsm_rough) * L.n);
    if (binned) {
        const int64_t key_bytes = precision == FSM_F64 ? 8 : 4;
        const int64_t per_item = (int64_t)fsm::kBlock * L.max_n;
        int64_t cap = bucket_cap(bucket_bytes, L.entry, per_item);
        cap = std::min<int64_t>(cap, std::max<int64_t>(per_item, bitems * per_item));
        L.per_slice = std::max<int64_t>(1, cap / per_item);
        L.per_slice = std::min<int64_t>(L.per_slice, std::max<int64_t>(1, bitems));
        L.cap = cap;
        const int64_t ht = L.total_htiles;
        const int64_t nb = ceil_div(ht, 4096);
        L.counts = take(sizeof(uint32_t) * ht);
        L.offsets = take(sizeof(uint32_t) * (ht + 1));
        L.cursor = take(sizeof(uint32_t) * ht);
        L.bsum = take(sizeof(uint32_t) * nb);
        L.bkey = take((size_t)key_bytes * cap);
        L.bidx = take(sizeof(uint16_t) * cap);
        if (L.super) {
            L.tile_lo = take(sizeof(uint32_t) * tiles);
            L.tile_hi = take(sizeof(uint32_t) * tiles);
            L.skey = take((size_t)key_bytes * cap);
            L.spk = take(sizeof(uint32_t) * cap);
        }
        if (L.hist) {
            // one slice when every item fits the bucket (the last row of a simulation may be
            // partial, so whole rows would overestimate); otherwise whole rows per slice
            const int64_t per_row = L.items_per_row * per_item;
            L.rows_per_slice = bitems * per_item <= cap ? L.total_rows : std::max<int64_t>(1, cap / per_row);
            L.rows_per_slice = std::min<int64_t>(L.rows_per_slice, std::max<int64_t>(1, L.total_rows));
            int64_t hsize = 0;
            for (const DevSim &d : devs) hsize += d.n_rows * d.h_tiles;
            L.hist_m = take(sizeof(uint32_t) * std::max<int64_t>(1, hsize));
            if (precision == FSM_F32) L.near_rows = take(sizeof(uint32_t) * std::max<int64_t>(1, L.total_rows));
            L.chunk = take(sizeof(uint32_t) * ceil_div(L.rows_per_slice, kRowChunk) * std::max<int64_t>(1, ht));
        }
    }
    L.scratch_end = o;
    L.sims = take(sizeof(DevSim) * L.n);
    L.ibase = take(sizeof(int64_t) * L.n);
    L.bbase = take(sizeof(int64_t) * L.n);
    L.tbase = take(sizeof(int64_t) * L.n);
    L.hbase = take(sizeof(int64_t) * L.n);
    L.gbase = take(sizeof(int64_t) * L.n);
    L.binned = take(sizeof(uint64_t) * L.n);
    L.evals = take(sizeof(int64_t) * L.n);
    L.near = take(sizeof(uint64_t) * L.n);
    // table sizes follow from the plan's shape, so a plan built without its tables lays out
    // the same image
    for (const Plan &P : plans) {
        const size_t pts = (size_t)P.z_n * P.N, angles = (size_t)P.z_n * P.S;
        L.pT.push_back(take(sizeof(double) * 3 * pts));
        L.pTf.push_back(take(sizeof(float) * 4 * pts));
        // only the precision's own angle table travels (it is per step in the fixed-step mode)
        L.cs.push_back(take(precision == FSM_F64 ? sizeof(double) * 2 * angles : 0));
        L.csf.push_back(take(precision == FSM_F32 ? sizeof(float) * 2 * angles : 0));
        L.gm.push_back(take(sizeof(double) * (size_t)P.z_n * P.n_groups));
    }
    L.total = o;
    return L;
}

bool fit_layout(const fsm_ctx *ctx, const std::vector<Plan> &plans, int precision,
                int64_t bytes, LaunchParams lp, SetLayout &L, std::vector<DevSim> &devs)
{
    for (int it = 0; it < 8; ++it) {
        devs.clear();
        L = make_layout(ctx, plans, precision, lp, devs);
        const int64_t entry = L.entry;
        if ((int64_t)L.total <= bytes) return true;
        const int64_t floor_bytes = (int64_t)fsm::kBlock * L.max_n * entry;
        const int64_t used = L.cap * entry;
        const int64_t next = used - ((int64_t)L.total - bytes) - (1 << 20);
        if (used <= floor_bytes) return false;
        lp.bucket_bytes = std::max(next, floor_bytes);
    }
    return false;
}

int ensure(fsm_ctx *ctx, Workspace &w, size_t dev_bytes, size_t host_bytes, size_t n_out)
{
    if (w.d_bytes < dev_bytes) {
        if (w.d_ws) {
            (void)hipFree(w.d_ws);
            if (&w == &ctx->ws) {
                // captured graphs point into the old workspace
                for (auto &g : ctx->graph_cache) (void)hipGraphExecDestroy(g.second);
                ctx->graph_cache.clear();
            }
        }
        w.d_ws = nullptr;
        w.d_bytes = 0;
        hipError_t e = hipMalloc(&w.d_ws, dev_bytes);
        if (e != hipSuccess) { w.d_ws = nullptr; return hip_err(ctx, e, "hipMalloc(workspace)"); }
        w.d_bytes = dev_bytes;
    }
    if (w.h_bytes < host_bytes) {
        if (w.h_ws) (void)hipHostFree(w.h_ws);
        w.h_ws = nullptr;
        w.h_bytes = 0;
        hipError_t e = hipHostMalloc(&w.h_ws, host_bytes, hipHostMallocDefault);
        if (e != hipSuccess) { w.h_ws = nullptr; return hip_err(ctx, e, "hipHostMalloc(staging)"); }
        w.h_bytes = host_bytes;
    }
    if (w.h_out_n < n_out) {
        if (w.h_out) (void)hipHostFree(w.h_out);
        w.h_out = nullptr;
        w.h_out_n = 0;
        hipError_t e = hipHostMalloc((void **)&w.h_out, sizeof(fsm_rough) * n_out, hipHostMallocDefault);
        if (e != hipSuccess) { w.h_out = nullptr; return hip_err(ctx, e, "hipHostMalloc(results)"); }
        w.h_out_n = n_out;
    }
    return FSM_OK;
}

void release(Workspace &w)
{
    if (w.d_ws) (void)hipFree(w.d_ws);
    if (w.h_ws) (void)hipHostFree(w.h_ws);
    if (w.h_out) (void)hipHostFree(w.h_out);
    w = Workspace();
}

// Fill the uploaded part of the image (host offsets are relative to L.sims).
void fill_image(const SetLayout &L, const std::vector<Plan> &plans, std::vector<DevSim> &devs,
                const std::vector<void *> &zmaps, char *dev, char *host)
{
    auto H = [&](size_t off) { return host + (off - L.sims); };
    std::vector<int64_t> ib(L.n), bb(L.n), tb(L.n), hb(L.n), gb(L.n), ev(L.n), rbase(L.n);
    std::vector<uint64_t> zero(L.n, 0);
    // every simulation writes its own descriptor and table ranges of the staging image
    parallel_for(L.n, [&](int k) {
        const Plan &P = plans[k];
        DevSim &d = devs[k];
        d.pT = reinterpret_cast<const double *>(dev + L.pT[k]);
        d.pTf = reinterpret_cast<const float *>(dev + L.pTf[k]);
        d.cs = reinterpret_cast<const double *>(dev + L.cs[k]);
        d.csf = reinterpret_cast<const float *>(dev + L.csf[k]);
        d.gm = reinterpret_cast<const double *>(dev + L.gm[k]);
        d.zmap = zmaps[k];
        d.near = reinterpret_cast<uint64_t *>(dev + L.near) + k;
        // every row of the histogram mode writes its own count (indexed by global row)
        d.near_rows = L.near_rows ? reinterpret_cast<uint32_t *>(dev + L.near_rows) : nullptr;
        ib[k] = d.item_base;
        bb[k] = d.bitem_base;
        tb[k] = d.tile_base;
        hb[k] = d.h_base;
        gb[k] = d.tgroup_base;
        rbase[k] = d.row_base;
        ev[k] = P.n_evals;
        if (!P.pT.empty()) std::memcpy(H(L.pT[k]), P.pT.data(), sizeof(double) * P.pT.size());
        float *pTf = reinterpret_cast<float *>(H(L.pTf[k]));
        for (size_t q = 0; q < (size_t)P.z_n * P.N && 3 * q + 2 < P.pT.size(); ++q) {
            pTf[4 * q] = (float)P.pT[3 * q];
            pTf[4 * q + 1] = (float)P.pT[3 * q + 1];
            pTf[4 * q + 2] = (float)P.pT[3 * q + 2];
            pTf[4 * q + 3] = 0.0f;
        }
        if (L.precision == FSM_F64) {
            if (!P.cs.empty()) std::memcpy(H(L.cs[k]), P.cs.data(), sizeof(double) * P.cs.size());
        } else {
            float *csf = reinterpret_cast<float *>(H(L.csf[k]));
            for (size_t q = 0; q < P.cs.size(); ++q) csf[q] = (float)P.cs[q];
        }
        if (!P.gm.empty()) std::memcpy(H(L.gm[k]), P.gm.data(), sizeof(double) * P.gm.size());
    });
    std::memcpy(H(L.sims), devs.data(), sizeof(DevSim) * L.n);
    std::memcpy(H(L.ibase), ib.data(), sizeof(int64_t) * L.n);
    std::memcpy(H(L.bbase), (L.hist ? rbase : bb).data(), sizeof(int64_t) * L.n);
    std::memcpy(H(L.tbase), tb.data(), sizeof(int64_t) * L.n);
    std::memcpy(H(L.hbase), hb.data(), sizeof(int64_t) * L.n);
    std::memcpy(H(L.gbase), gb.data(), sizeof(int64_t) * L.n);
    std::memcpy(H(L.binned), zero.data(), sizeof(uint64_t) * L.n);
    std::memcpy(H(L.evals), ev.data(), sizeof(int64_t) * L.n);
    std::memcpy(H(L.near), zero.data(), sizeof(uint64_t) * L.n);
}

void mark(fsm_ctx *ctx, int k, hipStream_t s, bool capturing)
{
    if (ctx->profiling && !capturing) (void)hipEventRecord(ctx->ev[k], s);
}

// Stage events of binned slice k of a profiled eager call (nullptr otherwise).
const fsm::StageEvents *stage_marks(fsm_ctx *ctx, size_t k, bool capturing)
{
    if (!ctx->profiling || capturing) return nullptr;
    while (ctx->stage_ev.size() <= k) {
        fsm::StageEvents m = {};
        for (void *&e : m.ev) {
            hipEvent_t h = nullptr;
            if (hipEventCreate(&h) != hipSuccess) return nullptr;
            e = h;
        }
        ctx->stage_ev.push_back(m);
    }
    ctx->stages_used = (int)k + 1;
    return &ctx->stage_ev[k];
}

// Read the events of a finished call into ctx->timings (phases that did not run read 0).
void collect(fsm_ctx *ctx, bool phases)
{
    if (!ctx->profiling) return;
    float t[4] = {0, 0, 0, 0};
    if (phases)
        for (int k = 0; k < 4; ++k)
            if (hipEventElapsedTime(&t[k], ctx->ev[k], ctx->ev[k + 1]) != hipSuccess) t[k] = 0.0f;
    ctx->timings.upload_ms = t[0];
    ctx->timings.fill_ms = t[1];
    ctx->timings.scatter_ms = t[2];
    ctx->timings.rough_ms = t[3];
    float st[4] = {0, 0, 0, 0};
    for (int k = 0; phases && k < ctx->stages_used; ++k)
        for (int j = 0; j < 4; ++j) {
            float v = 0.0f;
            if (hipEventElapsedTime(&v, static_cast<hipEvent_t>(ctx->stage_ev[k].ev[j]),
                                    static_cast<hipEvent_t>(ctx->stage_ev[k].ev[j + 1])) == hipSuccess)
                st[j] += v;
        }
    ctx->timings.count_ms = st[0];
    ctx->timings.index_ms = st[1];
    ctx->timings.write_ms = st[2];
    ctx->timings.reduce_ms = st[3];
    ctx->timings.n_slices = phases ? ctx->stages_used : 0;
    ctx->timings.zmap_path = ctx->zmap_path;
    float tot = 0.0f;
    if (hipEventElapsedTime(&tot, ctx->ev[0], ctx->ev[4]) != hipSuccess) tot = 0.0f;
    ctx->timings.total_ms = tot;
    ctx->timings.valid = 1;
}

// Every kernel of one set launch, in order (the part a graph captures).
int launch_set(fsm_ctx *ctx, const SetLayout &L, const std::vector<DevSim> &devs,
               const std::vector<Plan> &plans, char *dev, hipStream_t s, bool capturing)
{
    const DevSim *d_sims = reinterpret_cast<const DevSim *>(dev + L.sims);
    const int64_t *d_ibase = reinterpret_cast<const int64_t *>(dev + L.ibase);
    const int64_t *d_bbase = reinterpret_cast<const int64_t *>(dev + L.bbase);
    const int64_t *d_tbase = reinterpret_cast<const int64_t *>(dev + L.tbase);
    const int64_t *d_hbase = reinterpret_cast<const int64_t *>(dev + L.hbase);
    const int64_t *d_gbase = reinterpret_cast<const int64_t *>(dev + L.gbase);
    uint64_t *d_binned = reinterpret_cast<uint64_t *>(dev + L.binned);
    const int64_t *d_evals = reinterpret_cast<const int64_t *>(dev + L.evals);
    auto *st1 = reinterpret_cast<fsm::TileStat1 *>(dev + L.st1);
    auto *st2 = reinterpret_cast<fsm::TileStat2 *>(dev + L.st2);
    auto *state = reinterpret_cast<fsm::RoughState *>(dev + L.state);
    auto *d_out = reinterpret_cast<fsm_rough *>(dev + L.out);
    const bool binned = L.strategy == fsm::kStrategyBinned;
    ctx->zmap_path = !binned ? FSM_PATH_SCATTER : !L.hist ? FSM_PATH_RUN : L.super ? FSM_PATH_SUPER : FSM_PATH_HIST;
    int he = 0;
    mark(ctx, 1, s, capturing);
    if (!binned) {
        int64_t max_cells = 0;
        for (const Plan &P : plans) max_cells = std::max<int64_t>(max_cells, P.nx * P.ny);
        he = fsm::launch_fill(d_sims, L.n, max_cells, L.precision, s);
        if (he) return hip_err(ctx, (hipError_t)he, "fill kernel");
    }
    mark(ctx, 2, s, capturing);
    if (binned) {
        fsm::BinBuffers bb;
        bb.counts = reinterpret_cast<uint32_t *>(dev + L.counts);
        bb.offsets = reinterpret_cast<uint32_t *>(dev + L.offsets);
        bb.cursor = reinterpret_cast<uint32_t *>(dev + L.cursor);
        bb.bsum = reinterpret_cast<uint32_t *>(dev + L.bsum);
        bb.bkey = dev + L.bkey;
        bb.bidx = reinterpret_cast<uint16_t *>(dev + L.bidx);
        bb.cap = L.cap;
        bb.tile0 = bb.htile0 = 0;
        // per-tile bucket bounds: the split pass writes them with super-tiles; otherwise a
        // tile's bucket ends where the next one starts
        bb.tile_lo = L.super ? reinterpret_cast<uint32_t *>(dev + L.tile_lo) : bb.offsets;
        bb.tile_hi = L.super ? reinterpret_cast<uint32_t *>(dev + L.tile_hi) : bb.offsets + 1;
        bb.skey = L.super ? static_cast<void *>(dev + L.skey) : nullptr;
        bb.spk = L.super ? reinterpret_cast<uint32_t *>(dev + L.spk) : nullptr;
        bb.hist = L.hist ? reinterpret_cast<uint32_t *>(dev + L.hist_m) : nullptr;
        bb.chunk = L.hist ? reinterpret_cast<uint32_t *>(dev + L.chunk) : nullptr;
        bb.max_tiles = (int32_t)L.max_tiles;
        bb.row_chunk = kRowChunk;
        ctx->stages_used = 0;
        size_t slice = 0;
        if (L.hist) {
            // d_bbase holds each simulation's first row in this mode.  A slice works on the
            // tiles of the simulations its rows belong to (every simulation has a row).
            auto sim_of_row = [&](int64_t r) {
                int lo = 0, hi = L.n - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) / 2;
                    if (devs[mid].row_base <= r) lo = mid; else hi = mid - 1;
                }
                return lo;
            };
            int64_t r0 = 0;
            do {
                const int64_t r1 = std::min<int64_t>(L.total_rows, r0 + L.rows_per_slice);
                const DevSim &da = devs[sim_of_row(r0)], &db = devs[sim_of_row(r1 - 1)];
                const int64_t t0 = da.tile_base;
                const int64_t h0 = da.h_base, h1 = db.h_base + db.h_tiles;
                const int64_t g0 = da.tgroup_base, g1 = db.tgroup_base + db.n_tgroups;
                fsm::BinBuffers bs = bb;
                bs.tile0 = t0;
                bs.htile0 = h0;
                bs.counts += h0;
                bs.offsets += h0;
                bs.cursor += h0;
                bs.tile_lo += L.super ? t0 : h0;
                bs.tile_hi += L.super ? t0 : h0;
                he = fsm::launch_hist_slice(d_sims, L.n, d_bbase, d_hbase, h1 - h0,
                                            d_gbase, g0, g1 - g0, r0, r1, bs, L.precision, L.sx,
                                            L.sy, st1, d_binned, s, stage_marks(ctx, slice++, capturing));
                if (he) return hip_err(ctx, (hipError_t)he, "binned Z-map kernels");
                r0 = r1;
            } while (r0 < L.total_rows);
        } else if (L.total_items == 0) {
            // nothing to bin: the maps are still initialised and the first pass still runs
            he = fsm::launch_binned_slice(d_sims, L.n, d_bbase, L.total_tiles, d_gbase, 0,
                                          L.total_groups, 0, 0, bb, true, true, L.precision, L.sx,
                                          L.sy, st1, d_binned, s, stage_marks(ctx, slice++, capturing));
            if (he) return hip_err(ctx, (hipError_t)he, "binned Z-map kernels");
        }
        for (int64_t b0 = 0; !L.hist && b0 < L.total_items; b0 += L.per_slice) {
            const int64_t nit = std::min<int64_t>(L.per_slice, L.total_items - b0);
            he = fsm::launch_binned_slice(d_sims, L.n, d_bbase, L.total_tiles, d_gbase, 0,
                                          L.total_groups, b0, nit, bb, b0 == 0, b0 + nit >= L.total_items,
                                          L.precision, L.sx, L.sy, st1, d_binned, s,
                                          stage_marks(ctx, slice++, capturing));
            if (he) return hip_err(ctx, (hipError_t)he, "binned Z-map kernels");
        }
    } else {
        he = fsm::launch_scatter(d_sims, L.n, d_ibase, L.total_items, L.precision, d_binned, s);
        if (he) return hip_err(ctx, (hipError_t)he, "scatter kernel");
    }
    mark(ctx, 3, s, capturing);
    he = fsm::launch_rough(d_sims, L.n, d_tbase, L.total_tiles, L.precision, L.sx, L.sy, !binned,
                           !binned, st1, st2, state, d_binned, d_evals, d_out, s);
    if (he) return hip_err(ctx, (hipError_t)he, "roughness kernels");
    return FSM_OK;
}

int enqueue_set(fsm_ctx *ctx, Workspace &w, const SetLayout &L, const std::vector<Plan> &plans,
                std::vector<DevSim> &devs, const std::vector<void *> &zmaps, hipStream_t s,
                bool profile)
{
    char *dev = static_cast<char *>(w.d_ws);
    char *host = static_cast<char *>(w.h_ws);
    fill_image(L, plans, devs, zmaps, dev, host);
    hipError_t e = hipMemcpyAsync(dev + L.sims, host, L.total - L.sims, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(plan)");
    // the profiling events are the context's: only the synchronous calls record them
    int rc = launch_set(ctx, L, devs, plans, dev, s, !profile);
    if (rc != FSM_OK) return rc;
    e = hipMemcpyAsync(w.h_out, dev + L.out, sizeof(fsm_rough) * L.n, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(result)");
    return FSM_OK;
}

// Plan, upload, launch and wait for a set of simulations; results to out[0..n).
int run_set(fsm_ctx *ctx, const std::vector<Plan> &plans, const std::vector<void *> &zmaps,
            int precision, fsm_rough *out, hipStream_t user)
{
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_err(ctx, e, "hipSetDevice");
    std::vector<DevSim> devs;
    const SetLayout L = make_layout(ctx, plans, precision, params_for(ctx, plans, precision), devs);
    Workspace &w = ctx->ws;
    int rc = ensure(ctx, w, L.total, L.total - L.sims, (size_t)L.n);
    if (rc != FSM_OK) return rc;
    char *dev = static_cast<char *>(w.d_ws);
    char *host = static_cast<char *>(w.h_ws);

    hipStream_t s = user;
    if (ctx->graphs) {
        // graphs are captured and replayed on the context's own stream, after the caller's
        if (!ctx->own) {
            e = hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_err(ctx, e, "hipStreamCreate");
            e = hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming);
            if (e != hipSuccess) return hip_err(ctx, e, "hipEventCreate");
        }
        e = hipEventRecord(ctx->join, user);
        if (e != hipSuccess) return hip_err(ctx, e, "hipEventRecord");
        e = hipStreamWaitEvent(ctx->own, ctx->join, 0);
        if (e != hipSuccess) return hip_err(ctx, e, "hipStreamWaitEvent");
        s = ctx->own;
    }
    ctx->timings.valid = 0;
    ctx->stages_used = 0;
    mark(ctx, 0, s, false);
    if (ctx->graphs) {
        fill_image(L, plans, devs, zmaps, dev, host);
        e = hipMemcpyAsync(dev + L.sims, host, L.total - L.sims, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(plan)");
        char key[256];
        std::snprintf(key, sizeof key, "%d/%d/%d/%lld/%lld/%lld/%lld/%d/%d/%d/%d/%lld/%lld/%p", L.precision,
                      L.strategy, L.n, (long long)L.total_tiles, (long long)L.total_items,
                      (long long)L.per_slice, (long long)L.cap, L.sx, L.sy, (int)L.hist, (int)L.super,
                      (long long)L.total_rows, (long long)L.rows_per_slice, w.d_ws);
        // every host value a captured launch bakes in follows from these: the grids (tiles,
        // fill sizes) and each simulation's item and row counts (the tile range of every
        // slice); map pointers and tables travel in the uploaded descriptors
        std::string k(key);
        for (int i = 0; i < L.n; ++i)
            k += "/" + std::to_string(plans[i].nx) + "x" + std::to_string(plans[i].ny) + ":" +
                 std::to_string(devs[i].n_items) + ":" + std::to_string(devs[i].n_bitems) + ":" +
                 std::to_string(devs[i].n_rows);
        auto it = ctx->graph_cache.find(k);
        if (it == ctx->graph_cache.end()) {
            e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_err(ctx, e, "hipStreamBeginCapture");
            rc = launch_set(ctx, L, devs, plans, dev, s, true);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(s, &g);
            if (rc != FSM_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
            if (e2 != hipSuccess) return hip_err(ctx, e2, "hipStreamEndCapture");
            hipGraphExec_t x = nullptr;
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_err(ctx, e, "hipGraphInstantiate");
            it = ctx->graph_cache.emplace(k, x).first;
        }
        mark(ctx, 1, s, false);
        e = hipGraphLaunch(it->second, s);
        if (e != hipSuccess) return hip_err(ctx, e, "hipGraphLaunch");
        mark(ctx, 2, s, false);
        mark(ctx, 3, s, false);
        e = hipMemcpyAsync(w.h_out, dev + L.out, sizeof(fsm_rough) * L.n, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(result)");
    } else {
        rc = enqueue_set(ctx, w, L, plans, devs, zmaps, s, true);
        if (rc != FSM_OK) return rc;
    }
    mark(ctx, 4, s, false);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
    collect(ctx, !ctx->graphs);
    if (out) std::memcpy(out, w.h_out, sizeof(fsm_rough) * L.n);
    return FSM_OK;
}

bool valid_precision(int p) { return p == FSM_F64 || p == FSM_F32; }

int check_job_maps(fsm_ctx *ctx, const std::vector<Plan> &plans, const std::vector<void *> &zmaps,
                   int precision)
{
    const uintptr_t key = precision == FSM_F64 ? sizeof(double) : sizeof(float);
    std::vector<fsm::Span> spans(zmaps.size());
    for (size_t k = 0; k < zmaps.size(); ++k) {
        const uintptr_t b = reinterpret_cast<uintptr_t>(zmaps[k]);
        spans[k] = {b, b + (uintptr_t)plans[k].nx * (uintptr_t)plans[k].ny * key, (int)k, false};
    }
    const std::pair<int, int> o = fsm::first_conflict(std::move(spans));
    if (o.first < 0) return FSM_OK;
    return set_err(ctx, FSM_EINVAL, "jobs " + std::to_string(std::min(o.first, o.second)) + " and " +
                                        std::to_string(std::max(o.first, o.second)) + ": Z-maps overlap");
}

int roughness_maps(fsm_ctx *ctx, const fsm_grid *grid, int precision, const std::vector<void *> &zmaps,
                   fsm_rough *out, hipStream_t s)
{
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_err(ctx, e, "hipSetDevice");
    const int n = (int)zmaps.size();
    // a set of pseudo-simulations carrying only the grid: the tiled roughness passes
    std::vector<Plan> plans((size_t)n);
    for (Plan &p : plans) {
        p.nx = grid->nx;
        p.ny = grid->ny;
        p.N = 1;
    }
    std::vector<DevSim> devs;
    LaunchParams lp;
    lp.strategy = fsm::kStrategyScatter;
    lp.tile_shape = ctx->tile_shape;
    const SetLayout L = make_layout(ctx, plans, precision, lp, devs);
    int rc = ensure(ctx, ctx->ws, L.total, L.total - L.sims, (size_t)n);
    if (rc != FSM_OK) return rc;
    char *dev = static_cast<char *>(ctx->ws.d_ws);
    char *host = static_cast<char *>(ctx->ws.h_ws);
    fill_image(L, plans, devs, zmaps, dev, host);
    ctx->timings.valid = 0;
    ctx->stages_used = 0;
    mark(ctx, 0, s, false);
    e = hipMemcpyAsync(dev + L.sims, host, L.total - L.sims, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(plan)");
    mark(ctx, 1, s, false);
    mark(ctx, 2, s, false);
    mark(ctx, 3, s, false);
    int he = fsm::launch_rough(reinterpret_cast<const DevSim *>(dev + L.sims), n,
                               reinterpret_cast<const int64_t *>(dev + L.tbase), L.total_tiles,
                               precision, L.sx, L.sy, true, false,
                               reinterpret_cast<fsm::TileStat1 *>(dev + L.st1),
                               reinterpret_cast<fsm::TileStat2 *>(dev + L.st2),
                               reinterpret_cast<fsm::RoughState *>(dev + L.state), nullptr, nullptr,
                               reinterpret_cast<fsm_rough *>(dev + L.out), s);
    if (he) return hip_err(ctx, (hipError_t)he, "roughness kernels");
    e = hipMemcpyAsync(ctx->ws.h_out, dev + L.out, sizeof(fsm_rough) * (size_t)n, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(result)");
    mark(ctx, 4, s, false);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
    collect(ctx, true);
    std::memcpy(out, ctx->ws.h_out, sizeof(fsm_rough) * (size_t)n);
    return FSM_OK;
}

}  // namespace rt
}  // namespace fsm

using namespace fsm::rt;
using fsm::parallel_for;
using fsm::DevSim;
using fsm::Plan;

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
        fsm_ctx probe;
        std::vector<Plan> one{P};
        std::vector<DevSim> devs;
        const SetLayout L = make_layout(&probe, one, precision, LaunchParams(), devs);
        out->workspace_bytes = (int64_t)L.total;
        out->zmap_path = !L.hist ? FSM_PATH_RUN : L.super ? FSM_PATH_SUPER : FSM_PATH_HIST;
        out->n_slices = (int32_t)std::max<int64_t>(
            1, L.hist ? ceil_div(L.total_rows, L.rows_per_slice) : ceil_div(L.total_items, L.per_slice));
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

int fsm_refine(const fsm_tool *tool, const fsm_cut *cut, const fsm_grid *grid, double spacing,
               fsm_tool *tool_out, fsm_cut *cut_out)
{
    if (!tool || !cut || !grid || !tool_out || !cut_out || !(spacing > 0.0) || !std::isfinite(spacing))
        return FSM_EINVAL;
    try {
        fsm_tool t = *tool;
        fsm_cut c = *cut;
        std::string err;
        Plan P;
        int rc = fsm::build_plan(t, c, *grid, P, err, false);
        if (rc != FSM_OK) return rc;
        // largest distance between neighbouring edge points of any tooth (tool frame)
        auto edge_gap = [](const Plan &Q) {
            double gap = 0.0;
            for (int K = 0; K < Q.z_n; ++K)
                for (int p = 0; p + 1 < Q.N; ++p) {
                    const double *a = &Q.pT[((size_t)K * Q.N + p) * 3], *b = a + 3;
                    const double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
                    gap = std::max(gap, std::sqrt(dx * dx + dy * dy + dz * dz));
                }
            return gap;
        };
        // the edge is sampled uniformly in its parameter, so the gap shrinks like 1/(N - 1)
        for (int it = 0; it < 16 && edge_gap(P) > spacing; ++it) {
            const double need = std::ceil((double)(t.n_edge - 1) * edge_gap(P) / spacing) + 1.0;
            if (!(need <= (double)FSM_MAX_EDGE)) return FSM_EINVAL;
            t.n_edge = std::max(t.n_edge + 1, (int)need);
            rc = fsm::build_plan(t, c, *grid, P, err, false);
            if (rc != FSM_OK) return rc;
        }
        if (edge_gap(P) > spacing) return FSM_EINVAL;
        // in one time step a point at distance r from the axis turns through a chord of at most
        // r times the step angle, and the tool centre advances by the feed per step
        double r_max = 0.0;
        for (size_t k = 0; k < P.pT.size() / 3; ++k)
            r_max = std::max(r_max, std::sqrt(P.pT[3 * k] * P.pT[3 * k] + P.pT[3 * k + 1] * P.pT[3 * k + 1]));
        if (c.time_mode == FSM_TIME_FIXED_DT) {
            const double n_rpm = (1000.0 * c.v_c) / (M_PI * t.D);
            const double omega = ((2.0 * M_PI) * n_rpm) / 60.0;
            const double v_f = (c.f_z * (double)t.n_teeth * n_rpm) / 60.0;
            c.dt = std::min(c.dt, spacing / (omega * r_max + v_f));
        } else {
            const double need = std::ceil((2.0 * M_PI * r_max + (double)t.n_teeth * c.f_z) / spacing);
            if (!(need <= (double)(1 << 24))) return FSM_EINVAL;
            c.steps_per_rev = std::max(c.steps_per_rev, (int)need);
        }
        c.n_steps = 0;
        rc = fsm::build_plan(t, c, *grid, P, err, false);
        if (rc != FSM_OK) return rc;
        *tool_out = t;
        *cut_out = c;
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
    // the fixed scratch of fsm_simulate_noalloc: its address on this device, once per device
    // (a failure is reported by that call, not here)
    (void)noalloc_setup(device);
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->max_lds = (size_t)lds;
    *out = c;
    return FSM_OK;
}

void fsm_ctx_destroy(fsm_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (auto &g : ctx->graph_cache) (void)hipGraphExecDestroy(g.second);
    for (auto &ev : ctx->ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto &m : ctx->stage_ev)
        for (void *e : m.ev)
            if (e) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    if (ctx->join) (void)hipEventDestroy(ctx->join);
    if (ctx->own) (void)hipStreamDestroy(ctx->own);
    release_async(ctx);
    release(ctx->ws);
    delete ctx;
}

int fsm_last_error(const fsm_ctx *ctx, char *buf, size_t n)
{
    if (!ctx || !buf || n == 0) return FSM_EINVAL;
    std::snprintf(buf, n, "%s", ctx->err.c_str());
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
    case FSM_OPT_GRAPHS:
        ctx->graphs = value != 0;
        return FSM_OK;
    case FSM_OPT_TILE_SHAPE:
        if (value != 0 && !(valid_tile_shape(ctx, FSM_F64, (int)value) || valid_tile_shape(ctx, FSM_F32, (int)value)))
            return set_err(ctx, FSM_EINVAL, "tile shape out of range");
        ctx->tile_shape = (int)value;
        return FSM_OK;
    case FSM_OPT_TARGET_ROWS:
        if (value != 0 && (value < 256 || value > 65536))
            return set_err(ctx, FSM_EINVAL, "target rows out of range");
        ctx->target_rows = value ? value : 4096;
        return FSM_OK;
    case FSM_OPT_AUTOTUNED:
        ctx->use_tuned = value != 0;
        return FSM_OK;
    case FSM_OPT_ASYNC_SLOTS:
        if (value < 1 || value > 16) return set_err(ctx, FSM_EINVAL, "asynchronous slots out of range 1..16");
        for (const auto &sl : ctx->async)
            if (sl.id) return set_err(ctx, FSM_EAGAIN, "asynchronous batches in flight");
        release_async(ctx);
        ctx->async_slots = (int)value;
        return FSM_OK;
    case FSM_OPT_HBM_BUDGET:
        if (value < 0) return set_err(ctx, FSM_EINVAL, "negative HBM budget");
        ctx->hbm_budget = value;
        return FSM_OK;
    case FSM_OPT_HIST_BYTES:
        if (value < 0) return set_err(ctx, FSM_EINVAL, "negative row matrix budget");
        ctx->hist_bytes = value;
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

int fsm_simulate(fsm_ctx *ctx, const fsm_tool *tool, const fsm_cut *cut, const fsm_grid *grid,
                 int precision, void *zmap_dev, fsm_rough *out, void *stream)
{
    if (!ctx) return FSM_EINVAL;
    if (!tool || !cut || !grid || !zmap_dev || !valid_precision(precision))
        return set_err(ctx, FSM_EINVAL, "null argument or invalid precision");
    try {
        std::vector<Plan> plans(1);
        std::string err;
        int rc = fsm::build_plan(*tool, *cut, *grid, plans[0], err, true);
        if (rc != FSM_OK) return set_err(ctx, rc, err);
        std::vector<void *> zmaps{zmap_dev};
        return run_set(ctx, plans, zmaps, precision, out, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

int fsm_trajectory(fsm_ctx *ctx, const fsm_tool *tool, const fsm_cut *cut, const fsm_grid *grid,
                   int precision, void *traj_dev, int32_t *index_dev, void *stream)
{
    if (!ctx) return FSM_EINVAL;
    if (!tool || !cut || !grid || !traj_dev || !valid_precision(precision))
        return set_err(ctx, FSM_EINVAL, "null argument or invalid precision");
    try {
        std::vector<Plan> plans(1);
        std::string err;
        int rc = fsm::build_plan(*tool, *cut, *grid, plans[0], err, true);
        if (rc != FSM_OK) return set_err(ctx, rc, err);
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return hip_err(ctx, e, "hipSetDevice");
        // the image of one simulation (descriptor and tables); no Z-map is touched
        LaunchParams lp;
        lp.strategy = fsm::kStrategyScatter;
        std::vector<DevSim> devs;
        const SetLayout L = make_layout(ctx, plans, precision, lp, devs);
        rc = ensure(ctx, ctx->ws, L.total, L.total - L.sims, 1);
        if (rc != FSM_OK) return rc;
        char *dev = static_cast<char *>(ctx->ws.d_ws);
        std::vector<void *> zmaps{nullptr};
        fill_image(L, plans, devs, zmaps, dev, static_cast<char *>(ctx->ws.h_ws));
        hipStream_t s = static_cast<hipStream_t>(stream);
        e = hipMemcpyAsync(dev + L.sims, ctx->ws.h_ws, L.total - L.sims, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(plan)");
        const int he = fsm::launch_trajectory(reinterpret_cast<const DevSim *>(dev + L.sims),
                                              devs[0].n_bitems, precision, traj_dev, index_dev, s);
        if (he) return hip_err(ctx, (hipError_t)he, "trajectory kernel");
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
        return FSM_OK;
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

int fsm_simulate_batch(fsm_ctx *ctx, int n, const fsm_job *jobs, int precision, fsm_rough *out,
                       void *stream)
{
    if (!ctx) return FSM_EINVAL;
    if (n < 1 || !jobs || !out || !valid_precision(precision))
        return set_err(ctx, FSM_EINVAL, "empty batch, null argument or invalid precision");
    try {
        std::vector<Plan> plans((size_t)n);
        std::vector<void *> zmaps((size_t)n);
        for (int k = 0; k < n; ++k) {
            const fsm_job &j = jobs[k];
            if (!j.tool || !j.cut || !j.grid || !j.zmap_dev)
                return set_err(ctx, FSM_EINVAL, "job " + std::to_string(k) + ": null pointer");
            zmaps[k] = j.zmap_dev;
        }
        // the host plans (tables included) are independent: build them on several threads
        std::vector<int> rcs((size_t)n, FSM_OK);
        std::vector<std::string> errs((size_t)n);
        parallel_for(n, [&](int k) {
            rcs[k] = fsm::build_plan(*jobs[k].tool, *jobs[k].cut, *jobs[k].grid, plans[k], errs[k], true);
        });
        for (int k = 0; k < n; ++k)
            if (rcs[k] != FSM_OK) return set_err(ctx, rcs[k], "job " + std::to_string(k) + ": " + errs[k]);
        int rc = check_job_maps(ctx, plans, zmaps, precision);
        if (rc != FSM_OK) return rc;
        return run_set(ctx, plans, zmaps, precision, out, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

int fsm_autotune(fsm_ctx *ctx, int n, const fsm_job *jobs, int precision, fsm_tune_result *out,
                 void *stream)
{
    if (!ctx) return FSM_EINVAL;
    if (n < 1 || !jobs || !out || !valid_precision(precision))
        return set_err(ctx, FSM_EINVAL, "empty job list, null argument or invalid precision");
    try {
        std::vector<Plan> plans((size_t)n);
        std::vector<void *> zmaps((size_t)n);
        for (int k = 0; k < n; ++k) {
            if (!jobs[k].tool || !jobs[k].cut || !jobs[k].grid || !jobs[k].zmap_dev)
                return set_err(ctx, FSM_EINVAL, "job " + std::to_string(k) + ": null pointer");
            zmaps[k] = jobs[k].zmap_dev;
        }
        std::vector<int> rcs((size_t)n, FSM_OK);
        std::vector<std::string> errs((size_t)n);
        parallel_for(n, [&](int k) {
            rcs[k] = fsm::build_plan(*jobs[k].tool, *jobs[k].cut, *jobs[k].grid, plans[k], errs[k], true);
        });
        for (int k = 0; k < n; ++k)
            if (rcs[k] != FSM_OK) return set_err(ctx, rcs[k], "job " + std::to_string(k) + ": " + errs[k]);
        int jrc = check_job_maps(ctx, plans, zmaps, precision);
        if (jrc != FSM_OK) return jrc;
        hipStream_t s = static_cast<hipStream_t>(stream);

        // the candidates run eagerly through the tuned-table slot of this class; the guard
        // puts the context back however the search ends
        const std::string key = tune_key(plans, precision);
        struct Guard {
            fsm_ctx *c;
            std::map<std::string, LaunchParams> tuned;
            bool use, graphs;
            ~Guard() { c->tuned = tuned; c->use_tuned = use; c->graphs = graphs; }
        };
        LaunchParams best;
        float best_ms = 0.0f, base_ms = 0.0f;
        int tried = 0;
        {
        Guard guard{ctx, ctx->tuned, ctx->use_tuned, ctx->graphs};
        ctx->use_tuned = true;
        ctx->graphs = false;
        // one warm-up call, then the fastest of at least three timed calls and of as many as
        // fill 20 ms (at most 64): short workloads need many to rise above the noise
        auto time_of = [&](const LaunchParams &lp, float &ms) -> int {
            ctx->tuned[key] = lp;
            double best = 1e300, total = 0.0;
            for (int rep = 0; rep < 65 && (rep < 4 || total < 20.0); ++rep) {
                const auto t0 = std::chrono::steady_clock::now();
                const int rc = run_set(ctx, plans, zmaps, precision, nullptr, s);
                if (rc != FSM_OK) return rc;
                const double el = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                if (rep > 0) {
                    best = std::min(best, el);
                    total += el;
                }
            }
            ms = (float)best;
            ++tried;
            return FSM_OK;
        };
        LaunchParams base;
        base.strategy = fsm::kStrategyBinned;
        base.tile_shape = 0;
        base.target_rows = 4096;
        base.bucket_bytes = ctx->bucket_bytes;
        base.hist_bytes = ctx->hist_bytes;
        int rc = time_of(base, base_ms);
        if (rc != FSM_OK) return rc;
        best = base;
        best_ms = base_ms;
        // 1. tile shape with the default rows
        static const int shapes[] = {0x55, 0x65, 0x56, 0x66, 0x75, 0x76, 0x67, 0x77, 0x86, 0x68,
                                     0x78, 0x87};
        for (int code : shapes) {
            int dsx = 0, dsy = 0;
            choose_tiles(ctx, precision, 0, dsx, dsy);
            if (!valid_tile_shape(ctx, precision, code) || code == ((dsx << 4) | dsy)) continue;
            LaunchParams lp = base;
            lp.tile_shape = code;
            float ms = 0.0f;
            rc = time_of(lp, ms);
            if (rc != FSM_OK) return rc;
            if (ms < best_ms) { best_ms = ms; best = lp; }
        }
        // 2. rows per launch with the best tile
        for (int64_t rows : {1024, 2048, 8192, 16384}) {
            LaunchParams lp = best;
            lp.target_rows = rows;
            float ms = 0.0f;
            rc = time_of(lp, ms);
            if (rc != FSM_OK) return rc;
            if (ms < best_ms) { best_ms = ms; best = lp; }
        }
        // 3. the global-atomic strategy with the best tile (its roughness tiles)
        {
            LaunchParams lp = best;
            lp.strategy = fsm::kStrategyScatter;
            float ms = 0.0f;
            rc = time_of(lp, ms);
            if (rc != FSM_OK) return rc;
            if (ms < best_ms) { best_ms = ms; best = lp; }
        }
        }
        ctx->tuned[key] = best;
        out->strategy = best.strategy == fsm::kStrategyScatter ? FSM_ZMAP_SCATTER : FSM_ZMAP_BINNED;
        int bsx = 0, bsy = 0;
        choose_tiles(ctx, precision, best.tile_shape, bsx, bsy);
        out->tile_shape = (bsx << 4) | bsy;
        out->target_rows = (int32_t)best.target_rows;
        out->n_tried = tried;
        out->best_ms = best_ms;
        out->default_ms = base_ms;
        return FSM_OK;
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

int fsm_tune_get(const fsm_ctx *ctx, fsm_tune_entry *out, int cap, int *n)
{
    if (!ctx || !n || cap < 0 || (cap > 0 && !out)) return FSM_EINVAL;
    int k = 0;
    for (const auto &e : ctx->tuned) {
        if (k < cap) {
            fsm_tune_entry &o = out[k];
            std::memset(&o, 0, sizeof o);
            std::snprintf(o.key, sizeof o.key, "%s", e.first.c_str());
            o.strategy = e.second.strategy == fsm::kStrategyScatter ? FSM_ZMAP_SCATTER : FSM_ZMAP_BINNED;
            o.tile_shape = e.second.tile_shape;
            o.target_rows = (int32_t)e.second.target_rows;
        }
        ++k;
    }
    *n = k;
    return FSM_OK;
}

int fsm_tune_set(fsm_ctx *ctx, const fsm_tune_entry *entries, int n)
{
    if (!ctx) return FSM_EINVAL;
    if (n < 0 || (n > 0 && !entries)) return set_err(ctx, FSM_EINVAL, "null entries");
    for (int k = 0; k < n; ++k) {
        const fsm_tune_entry &e = entries[k];
        const size_t len = strnlen(e.key, sizeof e.key);
        const bool shape_ok = e.tile_shape == 0 || valid_tile_shape(ctx, FSM_F64, e.tile_shape) ||
                              valid_tile_shape(ctx, FSM_F32, e.tile_shape);
        if (len == 0 || len == sizeof e.key || (e.strategy != FSM_ZMAP_BINNED && e.strategy != FSM_ZMAP_SCATTER) ||
            !shape_ok || e.target_rows < 256 || e.target_rows > 65536)
            return set_err(ctx, FSM_EINVAL, "tuning entry " + std::to_string(k) + " is invalid");
    }
    for (int k = 0; k < n; ++k) {
        const fsm_tune_entry &e = entries[k];
        LaunchParams lp;
        lp.strategy = e.strategy == FSM_ZMAP_SCATTER ? fsm::kStrategyScatter : fsm::kStrategyBinned;
        lp.tile_shape = e.tile_shape;
        lp.target_rows = e.target_rows;
        lp.bucket_bytes = ctx->bucket_bytes;
    lp.hist_bytes = ctx->hist_bytes;
        ctx->tuned[std::string(e.key, strnlen(e.key, sizeof e.key))] = lp;
    }
    return FSM_OK;
}

int fsm_roughness(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zmap_dev,
                  fsm_rough *out, void *stream)
{
    if (!ctx) return FSM_EINVAL;
    if (!grid || !zmap_dev || !out || !valid_precision(precision) || grid->nx < 1 || grid->ny < 1 ||
        grid->nx > INT32_MAX || grid->ny > INT32_MAX || grid->nx > INT64_MAX / grid->ny)
        return set_err(ctx, FSM_EINVAL, "invalid grid, pointer or precision");
    try {
        std::vector<void *> zmaps{const_cast<void *>(zmap_dev)};
        return fsm::rt::roughness_maps(ctx, grid, precision, zmaps, out, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

}  // extern "C"
