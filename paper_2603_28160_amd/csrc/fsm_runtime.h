// fsm_runtime.h -- the context and the launch machinery shared by the C ABI (fsm_api.cpp) and
// the serving loop (fsm_serve.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fsm_internal.h"

namespace fsm {
namespace rt {

// Device workspace, pinned host staging and pinned result records of one stream of work.
struct Workspace {
    void *d_ws = nullptr;
    size_t d_bytes = 0;
    void *h_ws = nullptr;
    size_t h_bytes = 0;
    fsm_rough *h_out = nullptr;
    size_t h_out_n = 0;
};

// Launch parameters of one set: strategy, tile shape (0: default), histogram rows per launch,
// bucket budget.
struct LaunchParams {
    int strategy = kStrategyBinned;
    int tile_shape = 0;
    int64_t target_rows = 4096;
    int64_t bucket_bytes = (int64_t)16 << 30;
    int64_t hist_bytes = (int64_t)1 << 30;   // row matrix of the histogram mode, at most
};

// Shape and layout of one launch over a set of simulations.
struct SetLayout {
    int n = 0, precision = 0, strategy = 0, sx = 7, sy = 6;
    int64_t total_tiles = 0, total_items = 0, per_slice = 0, cap = 0;
    int max_n = 1;
    // histogram mode of the binned strategy (no global atomics), with super-tiles when a
    // simulation has more tiles than a row histogram holds
    bool hist = false, super = false;
    int64_t total_rows = 0, rows_per_slice = 0, max_tiles = 0, items_per_row = 1;
    int64_t total_htiles = 0;   // histogram tiles (super-tiles, else tiles)
    int64_t total_groups = 0;   // tile groups of the reduction
    int64_t entry = 0;          // bucket bytes per point
    // device-only region
    size_t st1 = 0, st2 = 0, state = 0, out = 0, counts = 0, offsets = 0, cursor = 0, bsum = 0,
           bkey = 0, bidx = 0, hist_m = 0, chunk = 0, tile_lo = 0, tile_hi = 0, skey = 0, spk = 0,
           near_rows = 0;
    size_t scratch_end = 0;
    // uploaded region
    size_t sims = 0, ibase = 0, bbase = 0, tbase = 0, hbase = 0, gbase = 0, binned = 0, evals = 0,
           near = 0;
    std::vector<size_t> pT, pTf, cs, csf, gm;
    size_t total = 0;
};

// One slot of asynchronous batches (fsm_batch_submit): its own stream, workspace and events,
// and the host plans of the batch in flight (read by its uploads until it is waited for).
struct AsyncSlot {
    hipStream_t stream = nullptr;
    hipEvent_t start = nullptr, done = nullptr;
    Workspace ws;
    uint64_t id = 0;          // batch in flight, 0: free
    int n = 0;
    std::vector<Plan> plans;
    std::vector<DevSim> devs;
};

}  // namespace rt
}  // namespace fsm

struct fsm_ctx {
    int device = 0;
    std::string err;
    fsm::rt::Workspace ws;       // workspace of the synchronous calls
    bool profiling = false;
    hipEvent_t ev[5] = {};       // upload, fill, z-map, roughness, end
    std::vector<fsm::StageEvents> stage_ev;   // per binned slice: the five stage events
    int stages_used = 0;                      // slices of the last profiled call
    int zmap_path = 0;                        // FSM_PATH_* of the last launch
    fsm_timings timings = {};
    int strategy = fsm::kStrategyBinned;
    int64_t bucket_bytes = (int64_t)16 << 30;
    int64_t hist_bytes = (int64_t)1 << 30;    // FSM_OPT_HIST_BYTES
    bool graphs = false;
    int tile_shape = 0;          // FSM_OPT_TILE_SHAPE (0: default)
    int64_t target_rows = 4096;  // FSM_OPT_TARGET_ROWS
    bool use_tuned = true;       // FSM_OPT_AUTOTUNED
    std::map<std::string, fsm::rt::LaunchParams> tuned;   // per workload class (fsm_autotune)
    hipStream_t own = nullptr;   // stream used for graph capture and replay
    hipEvent_t join = nullptr;
    std::map<std::string, hipGraphExec_t> graph_cache;
    size_t max_lds = 65536;
    // asynchronous batches
    std::vector<fsm::rt::AsyncSlot> async;   // created on demand, at most async_slots
    int async_slots = 2;                     // FSM_OPT_ASYNC_SLOTS
    int64_t hbm_budget = 0;                  // FSM_OPT_HBM_BUDGET: slot workspaces, 0: no limit
    uint64_t next_batch = 1;
};


namespace fsm {
namespace rt {

int set_err(fsm_ctx *ctx, int code, const std::string &msg);
int hip_err(fsm_ctx *ctx, hipError_t e, const char *where);
bool valid_precision(int p);
// Layout of one launch over `plans` with parameters lp (its bucket budget bounds the bucket
// arrays; the work runs in slices beyond).
SetLayout make_layout(const fsm_ctx *ctx, const std::vector<Plan> &plans, int precision,
                      const LaunchParams &lp, std::vector<DevSim> &devs);
// Workload class of a set (the key of the autotuner's table) and the parameters a call on it
// uses: the context's options, or what fsm_autotune kept for the class.
std::string tune_key(const std::vector<Plan> &plans, int precision);
LaunchParams params_for(const fsm_ctx *ctx, const std::vector<Plan> &plans, int precision);
// Layout of a set whose whole workspace fits `bytes`: starting from lp, the bucket budget
// shrinks (more slices) until it does; false if even the smallest bucket does not fit.
bool fit_layout(const fsm_ctx *ctx, const std::vector<Plan> &plans, int precision,
                int64_t bytes, LaunchParams lp, SetLayout &L, std::vector<DevSim> &devs);
// The fixed device scratch of fsm_simulate_noalloc on `device` (fsm_noalloc.hip): its
// address is looked up once per device, with the device current (fsm_ctx_create does it).
int noalloc_setup(int device);
// Whether a tile shape code is valid for the precision (and the context's LDS).
bool valid_tile_shape(const fsm_ctx *ctx, int precision, int code);
// Grow w to at least the given sizes (device workspace, host staging, result records).
int ensure(fsm_ctx *ctx, Workspace &w, size_t dev_bytes, size_t host_bytes, size_t n_out);
void release(Workspace &w);
// Wait for and free every asynchronous slot of the context (fsm_async.cpp).
void release_async(fsm_ctx *ctx);
// FSM_EINVAL, naming two jobs, when Z-maps of one set share a byte (the set's launches write
// them all); plans[k] gives the size of zmaps[k].
int check_job_maps(fsm_ctx *ctx, const std::vector<Plan> &plans, const std::vector<void *> &zmaps,
                   int precision);
// Roughness of existing Z-maps (device pointers) of one grid, one launch sequence; waits for
// stream s and writes zmaps.size() records to out.
int roughness_maps(fsm_ctx *ctx, const fsm_grid *grid, int precision, const std::vector<void *> &zmaps,
                   fsm_rough *out, hipStream_t s);
// Upload the image of L from w's staging, launch every kernel and queue the copy of the
// result records into w.h_out, all on stream s; returns without waiting.  profile: record the
// context's timing events (synchronous calls only).
int enqueue_set(fsm_ctx *ctx, Workspace &w, const SetLayout &L, const std::vector<Plan> &plans,
                std::vector<DevSim> &devs, const std::vector<void *> &zmaps, hipStream_t s,
                bool profile);

}  // namespace rt
}  // namespace fsm
