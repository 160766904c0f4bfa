// fsm_internal.h -- types shared by the translation units of libfsm (host planner, kernels,
// C ABI).  Not part of the public interface.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fsm.h"

namespace fsm {

// Host-side plan of one simulation: the resolved path, the discretised edge and the tables
// the kernels read.  All values are computed in double precision with libm on the host, in a
// fixed operation order, so that the device only ever adds, subtracts and multiplies them.
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
    std::vector<double> xc;   // [n_steps] tool-centre x per step
};

// Validate and build the plan.  Returns FSM_OK or FSM_EINVAL with a message in `err`.
int build_plan(const fsm_tool &t, const fsm_cut &c, const fsm_grid &g, Plan &out,
               std::string &err, bool tables = true);

// Device-side description of one simulation (plain data, copied to device memory).
struct DevSim {
    const double *pT;        // [z_n][N][3]
    const float *pTf;        // [z_n][N][4] (x, y, z, pad) single-precision copy
    const double *cs;        // [z_n][S][2]
    const float *csf;        // [z_n][S][2]
    const double *xc;        // [n_steps]
    void *zmap;              // encoded keys during the scatter, heights afterwards
    double y_first, a_e;
    double x_lo, y_lo, inv_dd;
    double nx_d, ny_d;       // nx, ny as doubles for the in-grid test
    int64_t nx, ny;
    double tl_c, tl_s, ts_c, ts_s;
    int32_t tilt_lead, tilt_side;
    int32_t z_n, N, S;
    int32_t n_steps;
    int32_t n_passes;
    int32_t chunk;           // steps per work item
    int32_t n_chunks;        // work items per (pass, tooth)
    int32_t ppi, spi;        // edge points per step slot, steps in flight per block
    int64_t n_items;         // n_passes * n_chunks * z_n
    int64_t item_base;       // first global work item of this simulation
    // binned Z-map: the grid is cut into kTile x kTile cell tiles
    int32_t tiles_x, tiles_y;
    int32_t n_sblocks;       // step blocks of kBlock steps per (pass, tooth)
    int32_t pad0;
    int64_t n_bitems;        // n_passes * n_sblocks * z_n
    int64_t bitem_base;      // first global binning item of this simulation
    int64_t tile_base;       // first global tile of this simulation
};

// Reduction partials and results of the roughness kernels (device memory).
struct RoughPart1 {
    double sum, mn, mx;
    int64_t n;
};
struct RoughPart2 {
    double s1, s2, s3, s4;
};
struct RoughState {
    double mean;
    double row_mean, col_mean;
    int64_t n, n_row, n_col;
    double mn, mx;
};

constexpr int kBlock = 256;            // threads per block of every kernel
constexpr int kRoughBlocks = 1024;     // blocks of the roughness passes (fixed: determinism)
constexpr int kTileShift = 6;
constexpr int kTile = 1 << kTileShift; // cells per tile side of the binned Z-map
constexpr int kScanThreads = 1024;

// Z-map strategies
constexpr int kStrategyBinned = 0;     // bucket points by tile, reduce each tile in LDS
constexpr int kStrategyScatter = 1;    // global atomic min per point

// Buffers of the binned Z-map path (device memory).
struct BinBuffers {
    uint32_t *counts;        // [n_tiles]
    uint32_t *offsets;       // [n_tiles + 1]
    uint32_t *cursor;        // [n_tiles]
    void *bkey;              // [cap] int64 (FP64) or int32 (FP32) height keys
    uint16_t *bidx;          // [cap] cell index inside the tile
    int64_t cap;             // bucket capacity (points)
};

// Launch wrappers (fsm_kernels.hip).  All return a hipError_t as int.
int launch_fill(void *zmap, int64_t n, int precision, void *stream);
int launch_scatter(const DevSim *d_sims, const DevSim &h_sim0, int64_t n_items, int n_sims,
                   const int64_t *d_item_base, int precision, uint64_t *d_binned, void *stream);
int launch_rough(void *zmap, int64_t nx, int64_t ny, int precision, bool decode,
                 RoughPart1 *p1, RoughPart2 *p2, RoughState *st, fsm_rough *d_out,
                 const uint64_t *d_binned, int64_t n_evals, void *stream);
int launch_decode(void *zmap, int64_t n, int precision, void *stream);
// One slice of binning items [item_begin, item_begin + n_items) of the binned path:
// count -> scan -> bucket write -> per-tile LDS reduction into the Z-map.
int launch_binned_slice(const DevSim *d_sims, int n_sims, const int64_t *d_bitem_base,
                        const int64_t *d_tile_base, int64_t n_tiles, int64_t item_begin,
                        int64_t n_items, const BinBuffers &bb, bool first_slice,
                        int precision, uint64_t *d_binned, void *stream);

}  // namespace fsm
