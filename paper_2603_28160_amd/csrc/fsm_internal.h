// fsm_internal.h -- types shared by the translation units of libfsm (host planner, kernels,
// C ABI).  Not part of the public interface.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <exception>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/fsm.h"

namespace fsm {

// Host-side plan of one simulation: the resolved path, the discretised edge and the tables
// the kernels read.  All values are computed in double precision with libm on the host, in a
// fixed operation order, so that the device only ever adds, subtracts, multiplies and (for the
// tool-centre position) divides them, each correctly rounded.
struct Plan {
    int kind = 0, z_n = 0, N = 0, S = 0;
    int64_t n_passes = 0, n_steps = 0, n_evals = 0;
    double r_reach = 0, x_start = 0, y_first = 0, a_e = 0;
    double x_lo = 0, y_lo = 0, inv_dd = 0;
    int64_t nx = 0, ny = 0;
    double tl_c = 1, tl_s = 0, ts_c = 1, ts_s = 0;   // tilt lead / side cos, sin
    bool tilt_lead = false, tilt_side = false;
    std::vector<double> pT;   // [z_n][N][3] tool-frame edge points
    std::vector<double> cs;   // [z_n][S][2] cos, sin of the spindle angle alpha
    // tool-centre x of step s (Eq. (4), feed along X): x_start + (s fpr) / S per revolution,
    // x_start + v_f (s dt) at a fixed time step; formed on the device in that order
    bool fixed_dt = false;
    double feed = 0, dt = 0;  // fpr (per revolution) or v_f (fixed step); dt
    // culling: per tooth and group of kGroup consecutive edge points, a radius that bounds
    // every point of the group around its reference point at any step
    int n_groups = 0;
    double x_hi = 0, y_hi = 0, cull_reach = 0;
    std::vector<double> gm;   // [z_n][n_groups]
    double pos_r = 0;         // largest distance of a tool-frame edge point from the origin
};

// Single-precision position error bound, in units of pos_r: the rotation, lead tilt and side
// tilt of a point in float with fused multiply-adds round at most 13 times per coordinate
// (inputs included), each error at most 2^-24 times a value no larger than pos_r in magnitude
// (every intermediate is a coordinate of a rotated edge point); 16 covers the second-order
// terms and the double-precision reference's own rounding.
constexpr double kF32PosErr = 16.0 / 16777216.0;

// Edge points per culling group, and the group's reference point (its middle point).
constexpr int kGroup = 16;
constexpr int group_ref(int g, int N)
{
    const int n = N - g * kGroup < kGroup ? N - g * kGroup : kGroup;
    return g * kGroup + n / 2;
}

// Validate and build the plan.  Returns FSM_OK or FSM_EINVAL with a message in `err`.
int build_plan(const fsm_tool &t, const fsm_cut &c, const fsm_grid &g, Plan &out,
               std::string &err, bool tables = true);

// Persistent host threads (up to 16 with the caller's, fsm_plan.cpp).  pool_run calls
// f(ctx, k) for k in [0, n) on them and on the calling thread and returns true; it returns
// false, having run nothing, when the pool is busy with another caller, when the caller is
// already inside a pool job (nested loops run inline), or in a process forked after the pool
// started.
bool pool_run(int n, void (*f)(void *, int), void *ctx);

// f(k) for k in [0, n) on the host pool (inline when it is unavailable); the first exception
// thrown by any f is rethrown here.
template <typename F>
void parallel_for(int n, F &&f)
{
    using Fn = std::remove_reference_t<F>;
    if (n >= 2) {
        struct Job {
            Fn *f;
            std::exception_ptr err;
            std::mutex m;
        } job{&f, nullptr, {}};
        auto call = [](void *p, int k) {
            Job &jb = *static_cast<Job *>(p);
            try {
                (*jb.f)(k);
            } catch (...) {
                std::lock_guard<std::mutex> g(jb.m);
                if (!jb.err) jb.err = std::current_exception();
            }
        };
        if (pool_run(n, call, &job)) {
            if (job.err) std::rethrow_exception(job.err);
            return;
        }
    }
    for (int k = 0; k < n; ++k) f(k);
}

constexpr int kRowChunk = 32;          // histogram rows per column-scan chunk
constexpr int kBlock = 256;            // threads per block of every kernel
constexpr int kWaves = kBlock / 64;    // waves per block

// Tile shapes of the binned Z-map and of the tiled roughness passes: (1 << sx) x (1 << sy)
// cells.  The keys of one tile live in LDS during the reduction (32 KiB: several blocks per
// compute unit).
inline int tile_sx(int precision) { return precision == FSM_F64 ? 6 : 7; }
inline int tile_sy(int precision) { (void)precision; return 6; }
// Largest per-simulation tile count whose per-block histogram fits in LDS (64 KiB).
constexpr int64_t kMaxHistTiles = 16384;
// Simulations with more tiles count their points per super-tile, a block of (1 << ux) x
// (1 << uy) tiles, so that a row histogram holds at most kSuperHistTiles counters (32 KiB,
// several blocks per compute unit); a split pass then sorts each super-tile's bucket into its
// tiles.  At most kMaxSubTiles tiles per super-tile.
constexpr int64_t kSuperHistTiles = 8192;
constexpr int kMaxSubShift = 6;
constexpr int kMaxSubTiles = 1 << kMaxSubShift;
// Tile groups of the reduction: as many tiles per group (a power of two, at most 64) as keep
// at least kReduceGroups groups per simulation; small maps reduce one tile per workgroup.
constexpr int64_t kReduceGroups = 2048;
constexpr int kMaxGroupShift = 6;

// Z-map strategies
constexpr int kStrategyBinned = 0;     // bucket points by tile, reduce each tile in LDS
constexpr int kStrategyScatter = 1;    // global atomic min per point

// Device-side description of one simulation (plain data, copied to device memory).
struct DevSim {
    const double *pT;        // [z_n][N][3]
    const float *pTf;        // [z_n][N][4] (x, y, z, pad) single-precision copy
    const double *cs;        // [z_n][S][2]
    const float *csf;        // [z_n][S][2]
    double x_start, feed, dt; // tool-centre x of step s: see centre_x
    int32_t fixed_dt, pad_c;
    void *zmap;              // the caller's Z-map
    double y_first, a_e;
    double x_lo, y_lo, inv_dd;
    double nx_d, ny_d;       // nx, ny as doubles for the in-grid test
    int64_t nx, ny;
    double tl_c, tl_s, ts_c, ts_s;
    int32_t tilt_lead, tilt_side;
    int32_t z_n, N, S;
    int32_t n_steps;
    int32_t n_passes;
    // scatter strategy: one item = (pass, chunk of steps, tooth), threads over edge points
    int32_t chunk;           // steps per item
    int32_t n_chunks;        // items per (pass, tooth)
    int32_t ppi, spi;        // edge points per step slot, steps in flight per block
    int64_t n_items;
    int64_t item_base;       // first global scatter item of this simulation
    // binned strategy: one item = (pass, block of kBlock steps, tooth), threads over steps
    int32_t n_sblocks;       // step blocks per (pass, tooth)
    int32_t pad0;
    int64_t n_bitems;        // n_passes * n_sblocks * z_n
    int64_t bitem_base;      // first global binning item of this simulation
    // tiles (binned Z-map and tiled roughness)
    int32_t sx, sy;          // tile = (1 << sx) x (1 << sy) cells
    int32_t tiles_x, tiles_y;
    int64_t n_tiles;
    int64_t tile_base;       // first global tile of this simulation
    int32_t sim;             // index of this simulation in its launch
    int32_t items_per_row;   // histogram binning: binning items per row
    int64_t n_rows;          // histogram binning: rows of this simulation
    int64_t row_base;        // first global row of this simulation
    int64_t hbase;           // offset of this simulation's first row in the row matrix
    // histogram tiles: the tiles themselves, or super-tiles of (1 << ux) x (1 << uy) tiles
    int32_t ux, uy;
    int32_t h_tiles_x;       // histogram tiles per grid row
    int32_t pad2;
    int64_t h_tiles;         // histogram tiles of this simulation (row width)
    int64_t h_base;          // first global histogram tile of this simulation
    // tile reduction: groups of (1 << tg_shift) consecutive tiles, one workgroup each, whose
    // first-pass partials are summed before a single block reduction
    int32_t tg_shift;
    int32_t pad3;
    int64_t n_tgroups;
    int64_t tgroup_base;     // first global tile group of this simulation
    // swept-box culling
    const double *gm;        // [z_n][n_groups] group radii
    int32_t n_groups;
    int32_t pad1;
    double x_hi, y_hi;       // upper grid boundaries
    double cull_reach;       // bound on any point's horizontal distance from the tool centre
    // single-precision error statement: the position error bound (mm, 0 in double precision),
    // the same in cell units widened for the binning arithmetic (< 0: none), and the counter
    // of in-grid evaluations that lay that close to a cell boundary
    double pos_err, near_w;
    uint64_t *near;
    // histogram mode: each row's count of those evaluations, indexed by global row (summed
    // with `near` into the result; nullptr in the other modes)
    uint32_t *near_rows;
};

// Per-tile partial sums of the roughness passes (device memory).  Row ny/2 and column nx/2
// carry the two profiles.
struct TileStat1 {
    double sum, mn, mx, row_sum, col_sum;
    int64_t n;
    int32_t row_n, col_n;
};
struct TileStat2 {
    double s1, s2, s3, s4, row_abs, col_abs;
};
struct RoughState {
    double mean, row_mean, col_mean, mn, mx;
    int64_t n, n_row, n_col;
};

// Buffers of the binned strategy (device memory).
struct BinBuffers {
    // counts, offsets and cursor are indexed by (global histogram tile - htile0), tile_lo and
    // tile_hi by (global tile - tile0): a slice of the histogram mode covers only the tiles of
    // the simulations its rows belong to.  Without super-tiles the histogram tiles are the
    // tiles, htile0 = tile0, and tile_lo / tile_hi are offsets / offsets + 1.
    int64_t tile0, htile0;
    uint32_t *counts;        // [n_htiles] points per histogram tile
    uint32_t *offsets;       // [n_htiles + 1] bucket starts
    uint32_t *cursor;        // [n_htiles] write cursors (run mode)
    uint32_t *bsum;          // [ceil(n_htiles / scan segment)] scan block sums
    uint32_t *tile_lo;       // [n_tiles] bucket of each tile: [tile_lo, tile_hi)
    uint32_t *tile_hi;
    void *bkey;              // [cap] int64 (FP64) or int32 (FP32) height keys
    uint16_t *bidx;          // [cap] cell index inside the tile
    int64_t cap;             // bucket capacity (points)
    // super-tiles: the write pass fills the super-tile buckets, whose cells carry the tile
    // inside the super-tile in their upper 16 bits; the split pass sorts them into bkey / bidx
    void *skey;              // [cap] keys, or nullptr without super-tiles
    uint32_t *spk;           // [cap] (tile inside the super-tile << 16) | cell inside the tile
    // histogram mode
    uint32_t *hist;          // row matrix: per row, the points of each tile of its simulation
    uint32_t *chunk;         // [n_chunks][n_tiles] column-scan partials
    int32_t max_tiles;       // largest tile count of a simulation in the launch
    int32_t row_chunk;       // rows per column-scan chunk
};

// Optional stage events of one binned slice (hipEvent_t handles, recorded on the launch
// stream): before counting, after counting, after the scans, after writing, after reducing.
struct StageEvents {
    void *ev[5];
};

// Launch wrappers (fsm_kernels.hip).  All return a hipError_t as int.  `sims`/`d_*base`
// describe n_sims simulations whose items and tiles are numbered consecutively.
// Every Z-map of the uploaded descriptors to +inf; max_cells: the largest map of the set.
int launch_fill(const DevSim *d_sims, int n_sims, int64_t max_cells, int precision, void *stream);
int launch_scatter(const DevSim *d_sims, int n_sims, const int64_t *d_item_base,
                   int64_t n_items, int precision, uint64_t *d_binned, void *stream);
// One slice [item_begin, item_begin + n_items) of binning items: count -> scan -> write ->
// per-tile LDS reduction into the Z-maps (with the first roughness pass on the last slice).
// Tiles are reduced in groups: d_gbase holds each simulation's first tile group, and the
// slice's tiles are the tile groups [g0, g0 + n_groups).
int launch_binned_slice(const DevSim *d_sims, int n_sims, const int64_t *d_bitem_base,
                        int64_t n_tiles, const int64_t *d_gbase, int64_t g0, int64_t n_groups,
                        int64_t item_begin, int64_t n_items,
                        const BinBuffers &bb, bool first_slice, bool last_slice, int precision,
                        int sx, int sy, TileStat1 *st1, uint64_t *d_binned, void *stream,
                        const StageEvents *marks = nullptr);
// Histogram mode of the binned strategy, one slice of rows [row_begin, row_end): per-block
// LDS histograms written as rows, a chunked column scan into per-(row, tile) offsets, a write
// pass that claims slots with LDS atomics only, then the per-tile LDS reduction.  The slice
// touches only the n_tiles tiles from bb.tile0 on (those of the simulations its rows belong
// to); a simulation's tiles are initialised in the slice holding its first row and their
// first roughness pass runs in the slice holding its last row.
// With super-tiles (bb.skey set) the histograms, scans and buckets are per super-tile
// (n_htiles of them from bb.htile0 on, simulations found through d_hbase) and a split pass
// sorts every super-tile's bucket into its tiles before the reduction.
int launch_hist_slice(const DevSim *d_sims, int n_sims, const int64_t *d_row_base,
                      const int64_t *d_hbase, int64_t n_htiles, const int64_t *d_gbase,
                      int64_t g0, int64_t n_groups,
                      int64_t row_begin, int64_t row_end, const BinBuffers &bb, int precision,
                      int sx, int sy, TileStat1 *st1, uint64_t *d_binned, void *stream,
                      const StageEvents *marks = nullptr);
// Trajectory module: per (pass, step, tooth) the lowest edge point's workpiece position.
int launch_trajectory(const DevSim *d_sim, int64_t n_items, int precision, void *traj,
                      int32_t *index, void *stream);
// Tiled roughness.  with_pass1: run the first pass (decoding scatter keys if `decode`);
// otherwise its tile partials are already in st1.  out: one record per simulation.
int launch_rough(const DevSim *d_sims, int n_sims, const int64_t *d_tile_base, int64_t n_tiles,
                 int precision, int sx, int sy, bool with_pass1, bool decode, TileStat1 *st1,
                 TileStat2 *st2, RoughState *state, const uint64_t *d_binned,
                 const int64_t *d_evals, fsm_rough *d_out, void *stream);

// Surface-texture operators (fsm_texture.hip), over n_maps maps of one grid at once: zin and
// zout are device arrays of n_maps map pointers (a map may be its own output).
// Least-squares plane over each map's hit cells, subtracted into its output, with nb blocks
// per map (plane_blocks gives a count for a batch size; any nb in [1, ny] works).  part:
// n_maps * nb * 9 doubles of scratch; coef: 4 doubles per map receiving (c0, cu, cv, status)
// in centred cell units.
constexpr int kPlanePartials = 1024 * 9;
int plane_blocks(int64_t ny, int n_maps);
int launch_plane(const void *const *zin, void *const *zout, int n_maps, int64_t nx, int64_t ny,
                 int precision, int nb, double *part, double *coef, void *stream);
// flag (device int) = 1 if any of the n cells of any map is empty, else 0.
int launch_scan_holes(const void *const *zin, int n_maps, int64_t n, int precision, int *flag, void *stream);
// Separable normalised Gaussian of half-width R cells: g_row holds K8 (2R + 1 rounded up to a
// multiple of 8) row weights, g_col 2R + 33 column weights (16 zeros on either side), nd
// 16 * nx * ny bytes of scratch per map.  holes = false asserts that every cell is hit: the
// denominators are then cx[i] cy[j] (nx and ny sums of the in-grid weights) and nd needs only
// 8 * nx * ny bytes per map.  mode 0: weighted mean; 1: input minus weighted mean.
int launch_gauss(const void *const *zin, void *const *zout, int n_maps, int64_t nx, int64_t ny, int precision,
                 int R, int K8, const double *g_row, const double *g_col, const double *cx, const double *cy,
                 bool holes, void *nd, int mode, void *stream);
// Dynamic LDS of the row pass for K8 row weights.
size_t gauss_lds_bytes(int K8);

}  // namespace fsm
