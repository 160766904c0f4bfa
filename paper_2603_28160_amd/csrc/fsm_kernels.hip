// fsm_kernels.hip -- gfx950 kernels of libfsm.
//
// The hot loop of the method (Sec. 2.3; the "surface computation" module of Sec. 3.2): every
// (pass, step, tooth, edge point) is turned into the workpiece frame on the fly (Eq. (3),
// tilt, Eq. (4)), binned into its half-open sampling boundary (Eq. (7)) and min-reduced into
// the Z-map.  Two strategies reach the Z-map:
//
//   scatter : one global integer atomic min per point on an order-preserving encoding of the
//             height.  Each point touches its own cache line of the map.
//   binned  : points are sorted by cell tile first and every tile is min-reduced in LDS.
//     histogram mode (default): a block owns a row of binning items.
//             count  - the row's points per tile in an LDS histogram, stored as the row's line
//                      of a row matrix;
//             index  - a chunked scan down the matrix's columns gives every (row, tile) its
//                      offset inside the tile's bucket;
//             write  - the row's points again; slots claimed with LDS atomics on the row's
//                      cursors, (height key, cell inside the tile) stored;
//             reduce - one block per group of consecutive tiles: keys in LDS, integer ds_min
//                      of every bucket entry, one coalesced store of each decoded tile, and the
//                      first roughness pass on the fly.
//     super mode: a map with more tiles than one histogram holds counts and writes per
//             super-tile (a block of tiles); a split pass then sorts every super-tile's bucket
//             into its tiles.
//     run mode: without room for a row matrix, counts and cursors are global atomics, one per
//             run of equal tiles in a wave (lanes are consecutive time steps).
//
// Roughness is tiled as well: per-tile (or per-group) partial sums (count, sum, min, max and
// the two profile lines; then the central moments), combined per simulation in a fixed order.
//
// Double precision: only +, -, * and the correctly rounded division of the tool-centre
// position run on the device (no contraction: -ffp-contract=off), in the order the host
// planner documents, so binning decisions equal those of the plain definition bit for bit.
// Single precision: rotation and tilt in float with explicit fused multiply-adds on
// tool-local coordinates; the tool-centre position, the binning (one double fused
// multiply-add per coordinate on the widened float offset) and the roughness moments stay in
// double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "fsm_internal.h"

namespace fsm {

namespace {

// Pointers that travel inside descriptors lose their address space; casting them back to
// the global address space lets the compiler emit global (not flat) loads and atomics.
#define FSM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ FSM_GLOBAL T *gptr(T *p) { return (FSM_GLOBAL T *)p; }

// Tool-centre x of step s (Eq. (4), feed along X) in the planner's operation order: the
// step's share of the feed per revolution, or the feed speed times the step's time.  Double
// division is correctly rounded on the device, so the position equals the plain definition's.
__device__ __forceinline__ double centre_x(const DevSim &d, int64_t s)
{
    return d.fixed_dt ? d.x_start + d.feed * ((double)s * d.dt)
                      : d.x_start + ((double)s * d.feed) / (double)d.S;
}

constexpr int64_t kInf64 = 0x7FF0000000000000LL;   // bits of +inf (double)
constexpr int32_t kInf32 = 0x7F800000;             // bits of +inf (float)

// Order-preserving map from IEEE heights to signed integers: non-negative values keep their
// bits, negative ones get every bit but the sign flipped.  The map is its own inverse.
__device__ __forceinline__ int64_t enc64(int64_t b) { return b >= 0 ? b : (b ^ 0x7FFFFFFFFFFFFFFFLL); }
__device__ __forceinline__ int32_t enc32(int32_t b) { return b >= 0 ? b : (b ^ 0x7FFFFFFF); }

template <int PREC> struct KeyOf;
template <> struct KeyOf<FSM_F64> {
    using T = int64_t;
    static constexpr int64_t inf = kInf64;
    __device__ static int64_t enc(int64_t k) { return enc64(k); }
    __device__ static double height(int64_t k) { return __longlong_as_double(k); }
};
template <> struct KeyOf<FSM_F32> {
    using T = int32_t;
    static constexpr int32_t inf = kInf32;
    __device__ static int32_t enc(int32_t k) { return enc32(k); }
    __device__ static double height(int32_t k) { return (double)__int_as_float(k); }
};
template <int PREC> __device__ __forceinline__ typename KeyOf<PREC>::T KT_inf() { return KeyOf<PREC>::inf; }

// 16-byte vectors of keys (two double keys or four float keys) for the tile fill and drain.
template <typename Key> struct KeyVec {
    static constexpr int n = 16 / (int)sizeof(Key);
    typedef Key T __attribute__((ext_vector_type(16 / sizeof(Key))));
};

// Block b of a launch runs on XCD (b mod 8).  Give every XCD a contiguous range of items so
// that the items sharing one XCD's L2 are neighbours along the tool path.
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t G)
{
    const int64_t g8 = G >> 3;
    if (b >= (g8 << 3)) return b;
    return (b & 7) * g8 + (b >> 3);
}

// Global item handled by block-loop index b of a grid-stride loop over n items.
__device__ __forceinline__ int64_t loop_item(int64_t b, int64_t n)
{
    const int64_t round0 = b - blockIdx.x;
    const int64_t rn = n - round0 < (int64_t)gridDim.x ? n - round0 : (int64_t)gridDim.x;
    return round0 + xcd_item(b - round0, rn);
}

// Work whose cost varies along the item order (binning rows: passes and steps far from the
// grid are culled) goes to the XCDs in interleaved chunks of kXcdChunk consecutive items, so
// every XCD gets a share of the heavy and the light parts while neighbouring items, which
// write into the same tiles' buckets, still share an L2.
constexpr int64_t kXcdChunk = 16;
__device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t G)
{
    const int64_t span = 8 * kXcdChunk;
    if (b >= G / span * span) return b;
    const int64_t k = b >> 3;
    return (k / kXcdChunk) * span + (b & 7) * kXcdChunk + (k % kXcdChunk);
}
__device__ __forceinline__ int64_t loop_chunk(int64_t b, int64_t n)
{
    const int64_t round0 = b - blockIdx.x;
    const int64_t rn = n - round0 < (int64_t)gridDim.x ? n - round0 : (int64_t)gridDim.x;
    return round0 + xcd_chunk(b - round0, rn);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide reduction of kBlock (= 4 waves) threads, valid in every thread.  Fixed order:
// lanes by butterfly, then waves 0..3 left to right.  `buf` holds 4 values.
template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, T *buf, Op op)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) buf[w] = v;
    __syncthreads();
    return op(op(buf[0], buf[1]), op(buf[2], buf[3]));
}
struct Add { template <typename T> __device__ T operator()(T a, T b) const { return a + b; } };
struct Min { __device__ double operator()(double a, double b) const { return fmin(a, b); } };
struct Max { __device__ double operator()(double a, double b) const { return fmax(a, b); } };

template <typename T>
__device__ __forceinline__ T block_sum(T v, T *buf) { return block_reduce(wave_sum(v), buf, Add()); }

// Index of the simulation owning global item / tile `x` (base ascending, base[0] == 0).
__device__ __forceinline__ int find_sim(const int64_t *__restrict__ base, int n, int64_t x)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

int stream_blocks(int64_t work, int64_t per_block, int cap)
{
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

constexpr int64_t kMaxGrid = (int64_t)1 << 20;

// Tiles with more keys than this run their reduction with eight waves per block.
constexpr size_t kTileLdsSmall = 65536;

// ---- fill ------------------------------------------------------------------------------------

// Every Z-map of a set starts at +inf (the scatter strategy min-reduces into it).  The map
// pointers come from the uploaded descriptors, so a captured launch fills the maps of the call
// that replays it.
template <typename K>
__global__ __launch_bounds__(kBlock) void fill_maps(const DevSim *__restrict__ sims, int n_sims, K inf)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int k = 0; k < n_sims; ++k) {
        FSM_GLOBAL K *z = gptr(static_cast<K *>(sims[k].zmap));
        const int64_t n = sims[k].nx * sims[k].ny;
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) z[i] = inf;
    }
}

__global__ __launch_bounds__(kBlock) void zero_u32(uint32_t *p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) p[k] = 0u;
}

// ---- kinematics of one point -----------------------------------------------------------------

// A tool-frame edge point and a spindle angle (cos, sin) in the kernel's precision.  Points are
// loaded once per edge point and reused over the lanes' steps.
template <int PREC> struct Edge;
template <> struct Edge<FSM_F64> { double x, y, z; };
template <> struct Edge<FSM_F32> { float x, y, z; };
template <int PREC> struct Turn;
template <> struct Turn<FSM_F64> { double c, s; };
template <> struct Turn<FSM_F32> { float c, s; };

template <int PREC>
__device__ __forceinline__ Edge<PREC> edge_point(const DevSim &d, int K, int p)
{
    Edge<PREC> e;
    if constexpr (PREC == FSM_F64) {
        const FSM_GLOBAL double *pt = gptr(d.pT + ((size_t)K * d.N + p) * 3);
        e.x = pt[0];
        e.y = pt[1];
        e.z = pt[2];
    } else {
        const FSM_GLOBAL float *pt = gptr(d.pTf + ((size_t)K * d.N + p) * 4);
        e.x = pt[0];
        e.y = pt[1];
        e.z = pt[2];
    }
    return e;
}

template <int PREC>
__device__ __forceinline__ Turn<PREC> spindle_turn(const DevSim &d, int K, int m)
{
    Turn<PREC> t;
    if constexpr (PREC == FSM_F64) {
        const FSM_GLOBAL double *cs = gptr(d.cs + ((size_t)K * d.S + m) * 2);
        t.c = cs[0];
        t.s = cs[1];
    } else {
        const FSM_GLOBAL float *cs = gptr(d.csf + ((size_t)K * d.S + m) * 2);
        t.c = cs[0];
        t.s = cs[1];
    }
    return t;
}

// Tilt modes: which of the two tilt rotations a simulation applies (bit 0 lead, bit 1 side).
// Kernels that walk many points pick the mode once per row and run a specialised loop; kTiltAny
// reads the flags per call.
constexpr int kTiltLead = 1, kTiltSide = 2, kTiltAny = -1;
__device__ __forceinline__ int tilt_mode(const DevSim &d)
{
    return (d.tilt_lead ? kTiltLead : 0) | (d.tilt_side ? kTiltSide : 0);
}

// Workpiece-frame horizontal offsets (xs, ys) of an edge point from the tool centre, and its
// height key.  Double precision: Eq. (3) [[c, s], [-s, c]] then the tilt rotations, in the
// oracle's operation order with no contraction.  Single precision: the same with fused
// multiply-adds.
template <int TILT = kTiltAny>
__device__ __forceinline__ void turn_point(const DevSim &d, const Turn<FSM_F64> &a,
                                           const Edge<FSM_F64> &e, double &xs, double &ys,
                                           int64_t &key)
{
    const bool lead = TILT == kTiltAny ? d.tilt_lead != 0 : (TILT & kTiltLead) != 0;
    const bool side = TILT == kTiltAny ? d.tilt_side != 0 : (TILT & kTiltSide) != 0;
    double x = a.c * e.x + a.s * e.y;
    double y = a.c * e.y - a.s * e.x;
    double z = e.z;
    if (lead) {
        const double x1 = d.tl_c * x + d.tl_s * z;
        z = d.tl_c * z - d.tl_s * x;
        x = x1;
    }
    if (side) {
        const double y1 = d.ts_c * y - d.ts_s * z;
        z = d.ts_s * y + d.ts_c * z;
        y = y1;
    }
    xs = x;
    ys = y;
    key = enc64(__double_as_longlong(z));
}
template <int TILT = kTiltAny>
__device__ __forceinline__ void turn_point(const DevSim &d, const Turn<FSM_F32> &a,
                                           const Edge<FSM_F32> &e, float &xs, float &ys,
                                           int32_t &key)
{
    const bool lead = TILT == kTiltAny ? d.tilt_lead != 0 : (TILT & kTiltLead) != 0;
    const bool side = TILT == kTiltAny ? d.tilt_side != 0 : (TILT & kTiltSide) != 0;
    float x = fmaf(a.c, e.x, a.s * e.y);
    float y = fmaf(a.c, e.y, -(a.s * e.x));
    float z = e.z;
    if (lead) {
        const float c = (float)d.tl_c, s = (float)d.tl_s;
        const float x1 = fmaf(c, x, s * z);
        z = fmaf(c, z, -(s * x));
        x = x1;
    }
    if (side) {
        const float c = (float)d.ts_c, s = (float)d.ts_s;
        const float y1 = fmaf(c, y, -(s * z));
        z = fmaf(s, y, c * z);
        y = y1;
    }
    xs = x;
    ys = y;
    key = enc32(__float_as_int(z));
}

// Eq. (4) tool-centre offset and Eq. (7) half-open sampling boundaries: the cell (i, j), or
// false outside the grid.  fx, fy: the position in cell units.
__device__ __forceinline__ bool bin_cell(const DevSim &d, double xcs, double yq, double xs,
                                         double ys, int32_t &i, int32_t &j, double &fx, double &fy)
{
    fx = ((xcs + xs) - d.x_lo) * d.inv_dd;
    fy = ((yq + ys) - d.y_lo) * d.inv_dd;
    if (fx >= 0.0 && fx < d.nx_d && fy >= 0.0 && fy < d.ny_d) {
        i = (int32_t)fx;
        j = (int32_t)fy;
        return true;
    }
    return false;
}

// One point of either precision: its cell (i, j) and key; false outside the grid.  Single
// precision turns the point in float on tool-local coordinates and widens the offsets to
// double; the position in cell units is then one double fused multiply-add per coordinate,
// (double)x_S / dd + (x_c - x_lo) / dd, whose second term is the same for every point of the
// step (a rounding of the order of 1e-11 cells away from the double-precision point's own
// formula).  near (single precision): the position lies within the error bound of a cell
// boundary, so double precision might bin it into a neighbour.
template <int TILT = kTiltAny>
__device__ __forceinline__ bool place_point(const DevSim &d, const Turn<FSM_F64> &a,
                                            const Edge<FSM_F64> &e, double xcs, double yq,
                                            int32_t &i, int32_t &j, int64_t &key, bool &near)
{
    double xs, ys, fx, fy;
    turn_point<TILT>(d, a, e, xs, ys, key);
    near = false;
    return bin_cell(d, xcs, yq, xs, ys, i, j, fx, fy);
}
template <int TILT = kTiltAny>
__device__ __forceinline__ bool place_point(const DevSim &d, const Turn<FSM_F32> &a,
                                            const Edge<FSM_F32> &e, double xcs, double yq,
                                            int32_t &i, int32_t &j, int32_t &key, bool &near)
{
    float xs, ys;
    turn_point<TILT>(d, a, e, xs, ys, key);
    // the step's centre in cell units: invariant over the step's edge points
    const double cx = (xcs - d.x_lo) * d.inv_dd, cy = (yq - d.y_lo) * d.inv_dd;
    const double fx = fma((double)xs, d.inv_dd, cx), fy = fma((double)ys, d.inv_dd, cy);
    const bool in = fx >= 0.0 && fx < d.nx_d && fy >= 0.0 && fy < d.ny_d;
    i = in ? (int32_t)fx : 0;
    j = in ? (int32_t)fy : 0;
    const double rx = fx - (double)i, ry = fy - (double)j, w = d.near_w;
    near = in && (rx < w || rx > 1.0 - w || ry < w || ry > 1.0 - w);
    return in;
}

// ---- culling -------------------------------------------------------------------------------------
//
// A wave of a binning item covers 64 consecutive steps of one pass and tooth.  Most of the
// auto path's evaluations land outside the grid (the path overshoots the grid by the tool
// reach on every side), so whole waves are skipped when the tool centre's path, widened by
// the reach, misses the grid, and then groups of kGroup edge points when no lane's disc around
// the group's reference point touches it.  The skipped points would have been dropped by the
// in-grid test, so results do not change.

// The steps of this thread's wave in step block sb: the first step, the last active lane and
// the tool-centre x at both ends (x grows with the step).  False past the pass's last step.
struct WaveSteps {
    int s0, last;
    double xc0, xc1;
};
__device__ __forceinline__ bool wave_steps(const DevSim &d, int sb, WaveSteps &w)
{
    const int s0 = __builtin_amdgcn_readfirstlane(sb * kBlock + (int)(threadIdx.x & ~63u));
    if (s0 >= d.n_steps) return false;
    const int rem = d.n_steps - 1 - s0;
    w.s0 = s0;
    w.last = rem < 63 ? rem : 63;
    w.xc0 = centre_x(d, s0);
    w.xc1 = centre_x(d, s0 + w.last);
    return true;
}

// False when the tool centre's path over the wave, widened by the reach, misses the grid.
__device__ __forceinline__ bool wave_near(const DevSim &d, const WaveSteps &w, double yq)
{
    return w.xc1 + d.cull_reach >= d.x_lo && w.xc0 - d.cull_reach < d.x_hi &&
           yq + d.cull_reach >= d.y_lo && yq - d.cull_reach < d.y_hi;
}

// False when no point of edge-point group g can land in the grid during the wave: every lane
// places the group's reference point at its own step, and every point of the group lies
// within the group's radius of it (the turn and tilts are rigid; the radius carries rounding
// slack), so a group whose discs around all active lanes' reference positions miss the grid
// has no point in the grid at any of the wave's steps.  Called in uniform control flow with
// every lane active; act: the lane holds one of the wave's steps.
template <int PREC, int TILT = kTiltAny>
__device__ __forceinline__ bool group_near(const DevSim &d, const Turn<PREC> &a,
                                           const Edge<PREC> &ref, int K, int g, double xcs,
                                           double yq, bool act)
{
    typename KeyOf<PREC>::T k;
    decltype(ref.x) fx, fy;
    turn_point<TILT>(d, a, ref, fx, fy, k);
    const double X = xcs + (double)fx, Y = yq + (double)fy;
    const double r = gptr(d.gm)[K * d.n_groups + g];
    const bool hit = act && X + r >= d.x_lo && X - r < d.x_hi && Y + r >= d.y_lo && Y - r < d.y_hi;
    return __ballot(hit) != 0;
}

// Add a wave's near-boundary counts to the simulation's counter (single precision; the
// scatter strategy and run mode: the histogram mode keeps one count per row instead).
__device__ __forceinline__ void add_near(const DevSim &d, uint32_t n)
{
    const uint32_t w = wave_sum(n);
    if ((threadIdx.x & 63) == 0 && w) atomicAdd((unsigned long long *)d.near, (unsigned long long)w);
}

// ---- scatter strategy ------------------------------------------------------------------------

template <int PREC>
__global__ __launch_bounds__(kBlock) void scatter(const DevSim *__restrict__ sims, int n_sims,
                                                  const int64_t *__restrict__ item_base,
                                                  int64_t n_items, uint64_t *__restrict__ binned)
{
    using KT = KeyOf<PREC>;
    using Key = typename KT::T;
    const int tid = threadIdx.x;
    for (int64_t b = blockIdx.x; b < n_items; b += gridDim.x) {
        const int64_t item = loop_item(b, n_items);
        const int si = n_sims == 1 ? 0 : find_sim(item_base, n_sims, item);
        const DevSim d = sims[si];
        int64_t local = item - d.item_base;
        const int K = (int)(local % d.z_n);
        local /= d.z_n;
        const int chunk = (int)(local % d.n_chunks);
        const int q = (int)(local / d.n_chunks);
        const int ppi = d.ppi, spi = d.spi;
        const int lane_p = tid % ppi, lane_s = tid / ppi;
        uint32_t cnt = 0, n_near = 0;
        if (lane_s < spi) {
            const int s0 = chunk * d.chunk;
            const int s1 = s0 + d.chunk < d.n_steps ? s0 + d.chunk : d.n_steps;
            const double yq = d.y_first + (double)q * d.a_e;
            const int S = d.S;
            FSM_GLOBAL Key *zk = gptr(static_cast<Key *>(d.zmap));
            for (int p = lane_p; p < d.N; p += ppi) {
                const Edge<PREC> e = edge_point<PREC>(d, K, p);
                int s = s0 + lane_s;
                int m = s % S;
                for (; s < s1; s += spi) {
                    const Turn<PREC> a = spindle_turn<PREC>(d, K, m);
                    const double xcs = centre_x(d, s);
                    Key key;
                    int32_t i, j;
                    bool near;
                    if (place_point(d, a, e, xcs, yq, i, j, key, near)) {
                        const int64_t idx = (int64_t)j * d.nx + i;
                        if (key < __hip_atomic_load(zk + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                            __hip_atomic_fetch_min(zk + idx, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ++cnt;
                        n_near += near;
                    }
                    m += spi;
                    while (m >= S) m -= S;
                }
            }
        }
        const uint32_t w = wave_sum(cnt);
        if ((tid & 63) == 0 && w) atomicAdd((unsigned long long *)(binned + d.sim), (unsigned long long)w);
        if (PREC == FSM_F32) add_near(d, n_near);
    }
}

// ---- trajectory module ---------------------------------------------------------------------------

// One item per (pass, block of kBlock steps, tooth), lanes over the steps: every lane walks the
// tooth's edge points and keeps the first one of least height (keys order like heights).
template <int PREC>
__global__ __launch_bounds__(kBlock) void trajectory(const DevSim *__restrict__ sims, int64_t n_items,
                                                     void *__restrict__ traj, int32_t *__restrict__ index)
{
    using Key = typename KeyOf<PREC>::T;
    using Real = decltype(Edge<PREC>::x);
    const DevSim d = sims[0];
    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        int64_t local = item;
        const int K = (int)(local % d.z_n);
        local /= d.z_n;
        const int sb = (int)(local % d.n_sblocks);
        const int q = (int)(local / d.n_sblocks);
        const int s = sb * kBlock + (int)threadIdx.x;
        if (s >= d.n_steps) continue;
        const Turn<PREC> a = spindle_turn<PREC>(d, K, s % d.S);
        Key best = KT_inf<PREC>();
        Real bx = 0, by = 0;
        int bp = -1;
        for (int p = 0; p < d.N; ++p) {
            Real xs, ys;
            Key key;
            turn_point(d, a, edge_point<PREC>(d, K, p), xs, ys, key);
            if (key < best) {
                best = key;
                bx = xs;
                by = ys;
                bp = p;
            }
        }
        const double xcs = centre_x(d, s);
        const double yq = d.y_first + (double)q * d.a_e;
        const int64_t o = ((int64_t)q * d.n_steps + s) * d.z_n + K;
        const double z = KeyOf<PREC>::height(KeyOf<PREC>::enc(best));
        if (PREC == FSM_F64) {
            FSM_GLOBAL double *t = gptr(static_cast<double *>(traj)) + 3 * o;
            t[0] = xcs + (double)bx;
            t[1] = yq + (double)by;
            t[2] = z;
        } else {
            FSM_GLOBAL float *t = gptr(static_cast<float *>(traj)) + 3 * o;
            t[0] = (float)(xcs + (double)bx);
            t[1] = (float)(yq + (double)by);
            t[2] = (float)z;
        }
        if (index) gptr(index)[o] = bp;
    }
}

// ---- binned strategy, run mode -------------------------------------------------------------------

constexpr int kUnroll = 4;   // edge points in flight per lane

struct Runs {
    bool head;               // first lane of a run of equal tiles
    int len;                 // run length (head lanes)
    int first;               // head lane of this lane's run
};

// Runs of equal tiles over the 64 lanes of a wave (t < 0: no tile).  Lanes hold consecutive
// time steps of one edge point, so a point's neighbours in time share its tile for a while.
__device__ __forceinline__ Runs tile_runs(int32_t t, int lane)
{
    Runs r;
    int32_t prev = __shfl_up(t, 1, 64);
    if (lane == 0) prev = -2;
    r.head = t >= 0 && t != prev;
    const uint64_t heads = __ballot(r.head);
    const uint64_t ends = heads | __ballot(t < 0);
    const uint64_t le = (2ull << lane) - 1ull;
    const uint64_t above = ends & ~le;
    const int nxt = above ? __ffsll((unsigned long long)above) - 1 : 64;
    r.len = nxt - lane;
    const uint64_t mine = heads & le;
    r.first = mine ? 63 - __clzll((long long)mine) : lane;
    return r;
}

// Counting (WRITE = false): one atomic add per run, its result unused.  Writing (WRITE =
// true): one atomic add per run on the tile's cursor claims the run's slots; every lane of the
// run stores (height key, cell inside the tile) at the head's slot plus its distance to it.
template <int PREC, bool WRITE>
__global__ __launch_bounds__(kBlock) void bin_points(const DevSim *__restrict__ sims, int n_sims,
                                                     const int64_t *__restrict__ bitem_base,
                                                     int64_t item_begin, int64_t n_items,
                                                     BinBuffers bb)
{
    using Key = typename KeyOf<PREC>::T;
    const int tid = threadIdx.x, lane = tid & 63;
    FSM_GLOBAL uint32_t *counter = gptr(WRITE ? bb.cursor : bb.counts);
    FSM_GLOBAL Key *bkey = gptr(static_cast<Key *>(bb.bkey));
    FSM_GLOBAL uint16_t *bix = gptr(bb.bidx);
    for (int64_t b = blockIdx.x; b < n_items; b += gridDim.x) {
        const int64_t item = item_begin + loop_chunk(b, n_items);
        const int si = n_sims == 1 ? 0 : find_sim(bitem_base, n_sims, item);
        const DevSim d = sims[si];
        int64_t local = item - d.bitem_base;
        const int K = (int)(local % d.z_n);
        local /= d.z_n;
        const int sb = (int)(local % d.n_sblocks);
        const int q = (int)(local / d.n_sblocks);
        WaveSteps w;
        if (!wave_steps(d, sb, w)) continue;
        const double yq = d.y_first + (double)q * d.a_e;
        if (!wave_near(d, w, yq)) continue;
        const bool vs = lane <= w.last;
        const int s = w.s0 + (vs ? lane : w.last);
        const Turn<PREC> a = spindle_turn<PREC>(d, K, s % d.S);
        const double xcs = centre_x(d, s);
        const int sx = d.sx, sy = d.sy;
        const int32_t mx = (1 << sx) - 1, my = (1 << sy) - 1;
        uint32_t n_near = 0;
        for (int g = 0; g < d.n_groups; ++g) {
            if (!group_near<PREC>(d, a, edge_point<PREC>(d, K, group_ref(g, d.N)), K, g, xcs, yq, vs)) continue;
            const int pg = g * kGroup;
            Edge<PREC> ep[kGroup];
#pragma unroll
            for (int u = 0; u < kGroup; ++u) ep[u] = edge_point<PREC>(d, K, pg + u < d.N ? pg + u : d.N - 1);
#pragma unroll
            for (int h = 0; h < kGroup; h += kUnroll) {
                int32_t tile[kUnroll];
                uint16_t cell[kUnroll];
                Key key[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    tile[u] = -1;
                    cell[u] = 0;
                    key[u] = 0;
                    if (vs && pg + h + u < d.N) {
                        int32_t i, j;
                        bool near;
                        if (place_point(d, a, ep[h + u], xcs, yq, i, j, key[u], near)) {
                            tile[u] = (int32_t)d.tile_base + (j >> sy) * d.tiles_x + (i >> sx);
                            cell[u] = (uint16_t)(((j & my) << sx) | (i & mx));
                            n_near += near;
                        }
                    }
                }
                Runs r[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) r[u] = tile_runs(tile[u], lane);
                if (!WRITE) {
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        if (r[u].head)
                            __hip_atomic_fetch_add(counter + tile[u], (uint32_t)r[u].len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    uint32_t base[kUnroll];
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u)
                        base[u] = r[u].head ? __hip_atomic_fetch_add(counter + tile[u], (uint32_t)r[u].len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
#pragma unroll
                    for (int u = 0; u < kUnroll; ++u) {
                        const uint32_t b0 = __shfl(base[u], r[u].first, 64);
                        if (tile[u] >= 0) {
                            const int64_t pos = (int64_t)b0 + (lane - r[u].first);
                            if (pos < bb.cap) {
                                bkey[pos] = key[u];
                                bix[pos] = cell[u];
                            }
                        }
                    }
                }
            }
        }
        if (!WRITE && PREC == FSM_F32) add_near(d, n_near);
    }
}

// ---- binned strategy, histogram mode ------------------------------------------------------------
//
// Without global atomics.  A block owns a row of consecutive binning items of one simulation
// and counts its points per tile in an LDS histogram over all tiles of that simulation; the
// histogram is stored as the row's entry of a row matrix.  A chunked column scan turns the
// matrix into the offset of every (row, tile) inside the tile's bucket, and the write pass
// recomputes the points, claiming slots with LDS atomics on the row's cursors.

// Visit every in-grid point of binning items [i0, i1) of simulation d: f(htile, cell, key,
// near) with the histogram tile numbered inside the simulation and the cell inside its tile;
// SUPER: the cell carries the tile inside the super-tile in its upper 16 bits.  Lanes hold
// the steps of a wave; the edge points of a culling group are loaded kBatch at a time ahead
// of their arithmetic.
constexpr int kBatch = 4;
template <int PREC, int TILT, bool SUPER, typename F>
__device__ __forceinline__ void row_points_tilt(const DevSim &d, int64_t i0, int64_t i1, F &f)
{
    using Key = typename KeyOf<PREC>::T;
    const int lane = threadIdx.x & 63;
    const int sx = d.sx, sy = d.sy, hsx = sx + d.ux, hsy = sy + d.uy;
    const int32_t mx = (1 << sx) - 1, my = (1 << sy) - 1;
    const int32_t mux = (1 << d.ux) - 1, muy = (1 << d.uy) - 1;
    const uint32_t htiles_x = (uint32_t)d.h_tiles_x;
    for (int64_t it = i0; it < i1; ++it) {
        int64_t local = it;
        const int K = (int)(local % d.z_n);
        local /= d.z_n;
        const int sb = (int)(local % d.n_sblocks);
        const int q = (int)(local / d.n_sblocks);
        WaveSteps w;
        if (!wave_steps(d, sb, w)) continue;
        const double yq = d.y_first + (double)q * d.a_e;
        if (!wave_near(d, w, yq)) continue;
        // the even steps of the wave go to lanes 0..31 and the odd ones to lanes 32..63, so
        // that neighbouring steps, which often share a tile, fall into different halves of
        // the wave's LDS accesses; lanes past the last step repeat it (they take part in the
        // culling test only)
        const int o = ((lane & 31) << 1) | (lane >> 5);
        const bool act = o <= w.last;
        const int s = w.s0 + (act ? o : w.last);
        const Turn<PREC> a = spindle_turn<PREC>(d, K, s % d.S);
        const double xcs = centre_x(d, s);
        for (int g = 0; g < d.n_groups; ++g) {
            if (!group_near<PREC, TILT>(d, a, edge_point<PREC>(d, K, group_ref(g, d.N)), K, g, xcs, yq, act)) continue;
            const int pg = g * kGroup;
            const int pe = pg + kGroup < d.N ? pg + kGroup : d.N;
            for (int p = pg; p < pe; p += kBatch) {
                Edge<PREC> e[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) e[u] = edge_point<PREC>(d, K, p + u < pe ? p + u : pe - 1);
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    Key key;
                    int32_t i, j;
                    bool near;
                    // the histogram tile is numbered inside the simulation; a histogram holds
                    // at most kMaxHistTiles tiles, so both factors fit the 24-bit multiply
                    if (p + u < pe && act && place_point<TILT>(d, a, e[u], xcs, yq, i, j, key, near)) {
                        uint32_t cell = (uint32_t)(((j & my) << sx) | (i & mx));
                        if constexpr (SUPER)
                            cell |= (uint32_t)((((j >> sy) & muy) << d.ux) | ((i >> sx) & mux)) << 16;
                        f((int32_t)(__umul24((uint32_t)(j >> hsy), htiles_x) + (uint32_t)(i >> hsx)),
                          cell, key, near);
                    }
                }
            }
        }
    }
}

// The same with the simulation's tilt mode fixed once for the row.
template <int PREC, bool SUPER, typename F>
__device__ __forceinline__ void row_points(const DevSim &d, int64_t i0, int64_t i1, F &&f)
{
    switch (tilt_mode(d)) {
    case 0: row_points_tilt<PREC, 0, SUPER>(d, i0, i1, f); break;
    case kTiltLead: row_points_tilt<PREC, kTiltLead, SUPER>(d, i0, i1, f); break;
    case kTiltSide: row_points_tilt<PREC, kTiltSide, SUPER>(d, i0, i1, f); break;
    default: row_points_tilt<PREC, kTiltLead | kTiltSide, SUPER>(d, i0, i1, f); break;
    }
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void hist_count(const DevSim *__restrict__ sims, int n_sims,
                                                     const int64_t *__restrict__ row_base,
                                                     int64_t r0, int64_t n_rows, BinBuffers bb)
{
    using Key = typename KeyOf<PREC>::T;
    extern __shared__ uint32_t hist[];
    const int tid = threadIdx.x;
    for (int64_t b = blockIdx.x; b < n_rows; b += gridDim.x) {
        const int64_t r = r0 + loop_chunk(b, n_rows);
        const int si = n_sims == 1 ? 0 : find_sim(row_base, n_sims, r);
        const DevSim d = sims[si];
        const int64_t lr = r - d.row_base;
        const int64_t i0 = lr * d.items_per_row;
        const int64_t i1 = i0 + d.items_per_row < d.n_bitems ? i0 + d.items_per_row : d.n_bitems;
        const int T = (int)d.h_tiles;
        for (int t = tid; t < T; t += kBlock) hist[t] = 0u;
        __syncthreads();
        uint32_t n_near = 0;
        row_points<PREC, false>(d, i0, i1, [&](int32_t lt, uint32_t, Key, bool near) {
            __hip_atomic_fetch_add(&hist[lt], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            n_near += near;
        });
        if (PREC == FSM_F32) {
            // the row's count in its own slot: no atomics on a shared counter
            __shared__ uint32_t wn[kWaves];
            const uint32_t w = wave_sum(n_near);
            if ((tid & 63) == 0) wn[tid >> 6] = w;
            __syncthreads();
            if (tid == 0) d.near_rows[r] = (wn[0] + wn[1]) + (wn[2] + wn[3]);
        }
        __syncthreads();
        FSM_GLOBAL uint32_t *row = gptr(bb.hist) + d.hbase + lr * T;
        for (int t = tid; t < T; t += kBlock) row[t] = hist[t];
        __syncthreads();
    }
}

// Rows of simulation d inside [lo, hi): clipped to its own rows.
__device__ __forceinline__ void sim_rows(const DevSim &d, int64_t lo, int64_t hi, int64_t &a, int64_t &b)
{
    a = lo > d.row_base ? lo : d.row_base;
    const int64_t e = d.row_base + d.n_rows;
    b = hi < e ? hi : e;
}

// Column sums of the row matrix over chunks of row_chunk rows of the slice [r0, r1), for the
// n_tiles tiles from bb.tile0 on.
__global__ __launch_bounds__(kBlock) void hist_colsum(const DevSim *__restrict__ sims, int n_sims,
                                                      const int64_t *__restrict__ tile_base,
                                                      int64_t n_tiles, int64_t r0, int64_t r1,
                                                      int64_t n_chunks, BinBuffers bb)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n_chunks * n_tiles; x += stride) {
        const int64_t c = x / n_tiles, t = bb.htile0 + (x - c * n_tiles);
        const int si = n_sims == 1 ? 0 : find_sim(tile_base, n_sims, t);
        const DevSim &d = sims[si];
        int64_t a, b;
        sim_rows(d, r0 + c * bb.row_chunk, r0 + (c + 1) * bb.row_chunk < r1 ? r0 + (c + 1) * bb.row_chunk : r1, a, b);
        const int64_t lt = t - d.h_base;
        uint32_t sum = 0;
        for (int64_t r = a; r < b; ++r) sum += bb.hist[d.hbase + (r - d.row_base) * d.h_tiles + lt];
        bb.chunk[x] = sum;
    }
}

// Exclusive scan of the chunk sums down every column; the column totals become the tile counts.
__global__ __launch_bounds__(kBlock) void hist_chunkscan(int64_t n_tiles, int64_t n_chunks, BinBuffers bb)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n_tiles; t += stride) {
        uint32_t run = 0;
        int64_t c = 0;
        // sixteen chunk sums in flight before their offsets are stored over them
        for (; c + 16 <= n_chunks; c += 16) {
            uint32_t v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = bb.chunk[(c + u) * n_tiles + t];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                bb.chunk[(c + u) * n_tiles + t] = run;
                run += v[u];
            }
        }
        for (; c < n_chunks; ++c) {
            const uint32_t v = bb.chunk[c * n_tiles + t];
            bb.chunk[c * n_tiles + t] = run;
            run += v;
        }
        bb.counts[t] = run;
    }
}

// Rows within a chunk: the matrix entries become offsets inside their tile's bucket.
__global__ __launch_bounds__(kBlock) void hist_apply(const DevSim *__restrict__ sims, int n_sims,
                                                     const int64_t *__restrict__ tile_base,
                                                     int64_t n_tiles, int64_t r0, int64_t r1,
                                                     int64_t n_chunks, BinBuffers bb)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x; x < n_chunks * n_tiles; x += stride) {
        const int64_t c = x / n_tiles, t = bb.htile0 + (x - c * n_tiles);
        const int si = n_sims == 1 ? 0 : find_sim(tile_base, n_sims, t);
        const DevSim &d = sims[si];
        int64_t a, b;
        sim_rows(d, r0 + c * bb.row_chunk, r0 + (c + 1) * bb.row_chunk < r1 ? r0 + (c + 1) * bb.row_chunk : r1, a, b);
        const int64_t lt = t - d.h_base;
        uint32_t run = bb.chunk[x];
        uint32_t *e = bb.hist + d.hbase + (a - d.row_base) * d.h_tiles + lt;
        const int64_t nr = b - a;
        if (nr == kRowChunk) {
            // the chunk's counts in flight before their offsets are stored over them
            uint32_t v[kRowChunk];
#pragma unroll
            for (int u = 0; u < kRowChunk; ++u) v[u] = e[(int64_t)u * d.h_tiles];
#pragma unroll
            for (int u = 0; u < kRowChunk; ++u) {
                e[(int64_t)u * d.h_tiles] = run;
                run += v[u];
            }
        } else {
            for (int64_t r = 0; r < nr; ++r) {
                const uint32_t v = e[r * d.h_tiles];
                e[r * d.h_tiles] = run;
                run += v;
            }
        }
    }
}

template <int PREC, bool SUPER>
__global__ __launch_bounds__(kBlock) void hist_write(const DevSim *__restrict__ sims, int n_sims,
                                                     const int64_t *__restrict__ row_base,
                                                     int64_t r0, int64_t n_rows, BinBuffers bb)
{
    using Key = typename KeyOf<PREC>::T;
    extern __shared__ uint32_t cur[];
    const int tid = threadIdx.x;
    FSM_GLOBAL Key *bkey = gptr(static_cast<Key *>(SUPER ? bb.skey : bb.bkey));
    FSM_GLOBAL uint16_t *bix = gptr(bb.bidx);
    FSM_GLOBAL uint32_t *spk = gptr(bb.spk);
    for (int64_t b = blockIdx.x; b < n_rows; b += gridDim.x) {
        const int64_t r = r0 + loop_chunk(b, n_rows);
        const int si = n_sims == 1 ? 0 : find_sim(row_base, n_sims, r);
        const DevSim d = sims[si];
        const int64_t lr = r - d.row_base;
        const int64_t i0 = lr * d.items_per_row;
        const int64_t i1 = i0 + d.items_per_row < d.n_bitems ? i0 + d.items_per_row : d.n_bitems;
        const int T = (int)d.h_tiles;
        const FSM_GLOBAL uint32_t *row = gptr(bb.hist) + d.hbase + lr * T;
        const FSM_GLOBAL uint32_t *off = gptr(bb.offsets) + (d.h_base - bb.htile0);
        for (int t = tid; t < T; t += kBlock) cur[t] = off[t] + row[t];
        __syncthreads();
        const int64_t cap = bb.cap;
        row_points<PREC, SUPER>(d, i0, i1, [&](int32_t lt, uint32_t cell, Key key, bool) {
            const uint32_t pos = __hip_atomic_fetch_add(&cur[lt], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if ((int64_t)pos < cap) {
                bkey[pos] = key;
                if constexpr (SUPER) spk[pos] = cell;
                else bix[pos] = (uint16_t)cell;
            }
        });
        __syncthreads();
    }
}

// A bucket [e0, e1) read in units of E neighbouring entries: the whole units [u0, u1) and at
// most E - 1 single entries at each end, [e0, hb) and [tb, e1).
struct UnitSplit {
    uint32_t e0, e1, u0, u1, hb, tb;
};
template <int E>
__device__ __forceinline__ UnitSplit unit_split(uint32_t e0, uint32_t e1)
{
    UnitSplit q;
    q.e0 = e0;
    q.e1 = e1;
    q.u0 = (e0 + E - 1) / E;
    q.u1 = e1 / E > q.u0 ? e1 / E : q.u0;
    q.hb = e1 < q.u0 * E ? e1 : q.u0 * E;
    q.tb = q.hb > q.u1 * E ? q.hb : q.u1 * E;
    if (q.tb > e1) q.tb = e1;   // no whole unit: the single entries end at e1
    return q;
}

// Super-tiles n_htiles from bb.htile0 on: sort each super-tile's bucket into the buckets of its
// tiles, in place of the same range of bkey / bidx, and write every tile's [tile_lo, tile_hi).
// One block per super-tile: an LDS count per tile inside the super-tile, their running sum,
// then a second read that claims slots with LDS atomics (the order inside a tile's bucket does
// not matter to its minimum).
constexpr int kSplitDepth = 2;   // units of four entries in flight per thread
template <int PREC>
__global__ __launch_bounds__(kBlock) void split_super(const DevSim *__restrict__ sims, int n_sims,
                                                      const int64_t *__restrict__ hbase,
                                                      int64_t n_htiles, BinBuffers bb)
{
    using Key = typename KeyOf<PREC>::T;
    __shared__ uint32_t cnt[kMaxSubTiles], cur[kMaxSubTiles];
    const int tid = threadIdx.x;
    const FSM_GLOBAL Key *skey = gptr(static_cast<const Key *>(bb.skey));
    const FSM_GLOBAL uint32_t *spk = gptr(bb.spk);
    FSM_GLOBAL Key *bkey = gptr(static_cast<Key *>(bb.bkey));
    FSM_GLOBAL uint16_t *bix = gptr(bb.bidx);
    typedef uint32_t P4 __attribute__((ext_vector_type(4)));
    typedef Key K4 __attribute__((ext_vector_type(4)));
    const FSM_GLOBAL P4 *upk = reinterpret_cast<const FSM_GLOBAL P4 *>(spk);
    const FSM_GLOBAL K4 *ukey = reinterpret_cast<const FSM_GLOBAL K4 *>(skey);
    const int64_t cap = bb.cap;
    for (int64_t b = blockIdx.x; b < n_htiles; b += gridDim.x) {
        const int64_t h = bb.htile0 + b;
        const int si = n_sims == 1 ? 0 : find_sim(hbase, n_sims, h);
        const DevSim &d = sims[si];
        const int64_t lh = h - d.h_base;
        const int stx = (int)(lh % d.h_tiles_x), sty = (int)(lh / d.h_tiles_x);
        const int ux = d.ux, nsub = 1 << (ux + d.uy);
        // entries past the capacity were never written; the clamp keeps the reads inside
        const uint32_t s0 = (int64_t)bb.offsets[b] < cap ? bb.offsets[b] : (uint32_t)cap;
        const uint32_t s1 = (int64_t)bb.offsets[b + 1] < cap ? bb.offsets[b + 1] : (uint32_t)cap;
        const uint32_t sm = (uint32_t)(nsub - 1);
        if (tid < nsub) cnt[tid] = 0u;
        __syncthreads();
        // both reads in units of four entries (the cells in one 16-byte load, the keys in one or
        // two), kSplitDepth units in flight per thread; single entries at the ends
        const UnitSplit q = unit_split<4>(s0, s1);
        const uint32_t nh = q.hb - q.e0, n1 = nh + (q.e1 - q.tb);
        const uint32_t eo = (uint32_t)tid < nh ? q.e0 + tid : q.tb + (tid - nh);   // thread's single entry
        uint32_t u = q.u0 + tid;
        for (; u + (kSplitDepth - 1) * kBlock < q.u1; u += kSplitDepth * kBlock) {
            P4 p[kSplitDepth];
#pragma unroll
            for (int v = 0; v < kSplitDepth; ++v) p[v] = __builtin_nontemporal_load(&upk[u + v * kBlock]);
#pragma unroll
            for (int v = 0; v < kSplitDepth; ++v)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    __hip_atomic_fetch_add(&cnt[(p[v][c] >> 16) & sm], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        for (; u < q.u1; u += kBlock) {
            const P4 p = __builtin_nontemporal_load(&upk[u]);
#pragma unroll
            for (int c = 0; c < 4; ++c)
                __hip_atomic_fetch_add(&cnt[(p[c] >> 16) & sm], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if ((uint32_t)tid < n1)
            __hip_atomic_fetch_add(&cnt[(spk[eo] >> 16) & sm], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
        if (tid == 0) {
            uint32_t run = s0;
            for (int k = 0; k < nsub; ++k) {
                cur[k] = run;
                run += cnt[k];
            }
        }
        __syncthreads();
        if (tid < nsub) {
            const int tx = (stx << ux) + (tid & ((1 << ux) - 1)), ty = (sty << d.uy) + (tid >> ux);
            if (tx < d.tiles_x && ty < d.tiles_y) {
                const int64_t t = d.tile_base + (int64_t)ty * d.tiles_x + tx - bb.tile0;
                bb.tile_lo[t] = cur[tid];
                bb.tile_hi[t] = cur[tid] + cnt[tid];
            }
        }
        __syncthreads();
        auto place = [&](Key k, uint32_t pk) {
            const uint32_t pos = __hip_atomic_fetch_add(&cur[(pk >> 16) & sm], 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
            bkey[pos] = k;
            bix[pos] = (uint16_t)pk;
        };
        u = q.u0 + tid;
        for (; u + (kSplitDepth - 1) * kBlock < q.u1; u += kSplitDepth * kBlock) {
            K4 k[kSplitDepth];
            P4 p[kSplitDepth];
#pragma unroll
            for (int v = 0; v < kSplitDepth; ++v) {
                k[v] = __builtin_nontemporal_load(&ukey[u + v * kBlock]);
                p[v] = __builtin_nontemporal_load(&upk[u + v * kBlock]);
            }
#pragma unroll
            for (int v = 0; v < kSplitDepth; ++v)
#pragma unroll
                for (int c = 0; c < 4; ++c) place(k[v][c], p[v][c]);
        }
        for (; u < q.u1; u += kBlock) {
            const K4 k = __builtin_nontemporal_load(&ukey[u]);
            const P4 p = __builtin_nontemporal_load(&upk[u]);
#pragma unroll
            for (int c = 0; c < 4; ++c) place(k[c], p[c]);
        }
        if ((uint32_t)tid < n1) place(skey[eo], spk[eo]);
        __syncthreads();
    }
}

// Exclusive scan of the tile counts in three launches: per-block sums of kScanSeg tiles, a
// one-block scan of those sums, and the per-block scan that writes offsets and cursors.
constexpr int kScanSeg = 4096;
constexpr int kScanPer = kScanSeg / kBlock;   // tiles per thread

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) sh[w] = x;
    __syncthreads();
    uint32_t wo = 0;
    for (int k = 0; k < w; ++k) wo += sh[k];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    return wo + x - v;
}

__global__ __launch_bounds__(kBlock) void scan_reduce(const uint32_t *counts, int64_t n, uint32_t *bsum)
{
    __shared__ uint32_t sh[4];
    const int64_t a = (int64_t)blockIdx.x * kScanSeg + (int64_t)threadIdx.x * kScanPer;
    uint32_t v = 0;
    for (int k = 0; k < kScanPer; ++k)
        if (a + k < n) v += counts[a + k];
    uint32_t tot;
    block_exclusive_scan(v, sh, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void scan_top(uint32_t *bsum, int nb, uint32_t *offsets, int64_t n)
{
    __shared__ uint32_t sh[4];
    uint32_t carry = 0;
    for (int c = 0; c < nb; c += kBlock) {
        const int k = c + threadIdx.x;
        const uint32_t v = k < nb ? bsum[k] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, sh, tot);
        if (k < nb) bsum[k] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) offsets[n] = carry;
}

__global__ __launch_bounds__(kBlock) void scan_apply(const uint32_t *counts, int64_t n, const uint32_t *bsum,
                                                    uint32_t *offsets, uint32_t *cursor)
{
    __shared__ uint32_t sh[4];
    const int64_t a = (int64_t)blockIdx.x * kScanSeg + (int64_t)threadIdx.x * kScanPer;
    uint32_t c[kScanPer];
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        c[k] = a + k < n ? counts[a + k] : 0u;
        v += c[k];
    }
    uint32_t tot;
    uint32_t run = bsum[blockIdx.x] + block_exclusive_scan(v, sh, tot);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (a + k < n) {
            offsets[a + k] = run;
            cursor[a + k] = run;
        }
        run += c[k];
    }
}

// The same for at most kScanSeg tiles in one block: offsets, cursors and the total.
__global__ __launch_bounds__(kBlock) void scan_single(const uint32_t *counts, int64_t n, uint32_t *offsets,
                                                     uint32_t *cursor)
{
    __shared__ uint32_t sh[4];
    const int64_t a = (int64_t)threadIdx.x * kScanPer;
    uint32_t c[kScanPer];
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        c[k] = a + k < n ? counts[a + k] : 0u;
        v += c[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(v, sh, tot);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (a + k < n) {
            offsets[a + k] = run;
            cursor[a + k] = run;
        }
        run += c[k];
    }
    if (threadIdx.x == 0) offsets[n] = tot;
}

// Accumulator of the first roughness pass over one tile or group of tiles.
struct Stat1Acc {
    double sum = 0.0, mn = INFINITY, mx = -INFINITY, row_sum = 0.0, col_sum = 0.0;
    int64_t n = 0;
    int32_t cnt = 0, row_n = 0, col_n = 0;   // cnt: cells counted by add / add_vec
    // One cell; +inf (not cut) counts nowhere.  Branch-free: an uncut cell adds 0 to the
    // sum, and +inf cannot lower the minimum.
    __device__ void add(double v, bool on_row, bool on_col)
    {
        const bool h = v < INFINITY;
        const double w = h ? v : 0.0;
        sum += w;
        mn = fmin(mn, v);
        mx = fmax(mx, h ? v : -INFINITY);
        cnt += h;
        if (on_row) { row_sum += w; row_n += h; }
        if (on_col) { col_sum += w; col_n += h; }
    }
    // V neighbouring cells of one map row (row_hit: the row is the feed profile; col_at: the
    // index among them of the pick profile's column, or -1): their sum joins the running sum
    // as one term, which shortens the dependency chain.
    template <int V>
    __device__ void add_vec(const double (&v)[V], bool row_hit, int col_at)
    {
        double w[V];
#pragma unroll
        for (int c = 0; c < V; ++c) {
            const bool h = v[c] < INFINITY;
            w[c] = h ? v[c] : 0.0;
            mn = fmin(mn, v[c]);
            mx = fmax(mx, h ? v[c] : -INFINITY);
            cnt += h;
        }
        double t;
        if constexpr (V == 2) t = w[0] + w[1];
        else if constexpr (V == 4) t = (w[0] + w[1]) + (w[2] + w[3]);
        else {
            t = w[0];
#pragma unroll
            for (int c = 1; c < V; ++c) t += w[c];
        }
        sum += t;
        if (row_hit) {
            row_sum += t;
#pragma unroll
            for (int c = 0; c < V; ++c) row_n += v[c] < INFINITY;
        }
        if (col_at >= 0) {
#pragma unroll
            for (int c = 0; c < V; ++c)
                if (c == col_at) { col_sum += w[c]; col_n += v[c] < INFINITY; }
        }
    }
    // Block totals in every thread of a block of NW waves: butterflies within each wave, then
    // the waves' partials by a pairwise tree in wave order (for four waves, the order of
    // block_reduce), with one barrier for all eight values.
    // This thread's values as a partial (an empty one for a fresh accumulator).
    __device__ TileStat1 partial() const
    {
        TileStat1 t;
        t.sum = sum;
        t.mn = mn;
        t.mx = mx;
        t.row_sum = row_sum;
        t.col_sum = col_sum;
        t.n = n + cnt;
        t.row_n = row_n;
        t.col_n = col_n;
        return t;
    }
    // rows / cols (uniform over the block): whether any thread may hold cells of the feed /
    // pick profile (every thread's profile terms are zero otherwise, and their sums are
    // skipped); tile: the accumulator holds one tile's cells, whose count fits 32 bits.
    template <int NW = kWaves>
    __device__ TileStat1 reduce(bool rows = true, bool cols = true, bool tile = false)
    {
        static_assert(NW == 4 || NW == 8, "four or eight waves");
        __shared__ double bd[5][8];
        __shared__ int64_t bl[8];
        __shared__ int32_t bi[2][8];
        const int w = threadIdx.x >> 6;
        const double s0 = wave_sum(sum), s1 = wave_min(mn), s2 = wave_max(mx);
        const double s3 = rows ? wave_sum(row_sum) : 0.0, s4 = cols ? wave_sum(col_sum) : 0.0;
        const int64_t c0 = tile ? (int64_t)wave_sum(cnt) : wave_sum(n + (int64_t)cnt);
        const int32_t c1 = rows ? wave_sum(row_n) : 0, c2 = cols ? wave_sum(col_n) : 0;
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
            bd[0][w] = s0;
            bd[1][w] = s1;
            bd[2][w] = s2;
            bd[3][w] = s3;
            bd[4][w] = s4;
            bl[w] = c0;
            bi[0][w] = c1;
            bi[1][w] = c2;
        }
        __syncthreads();
        TileStat1 t;
        t.sum = tree<NW>(bd[0], Add());
        t.mn = tree<NW>(bd[1], Min());
        t.mx = tree<NW>(bd[2], Max());
        t.row_sum = tree<NW>(bd[3], Add());
        t.col_sum = tree<NW>(bd[4], Add());
        t.n = tree<NW>(bl, Add());
        t.row_n = tree<NW>(bi[0], Add());
        t.col_n = tree<NW>(bi[1], Add());
        return t;
    }
    template <int NW, typename T, typename Op>
    __device__ static T tree(const T *v, Op op)
    {
        const T a = op(op(v[0], v[1]), op(v[2], v[3]));
        if constexpr (NW == 4) return a;
        else return op(a, op(op(v[4], v[5]), op(v[6], v[7])));
    }
};

// Geometry of tile t of simulation d: origin (i0, j0) and extent w x h (ragged at the edges).
struct TileGeom {
    int64_t i0, j0;
    int w, h;
};
__device__ __forceinline__ TileGeom tile_geom(const DevSim &d, int64_t t)
{
    const int64_t lt = t - d.tile_base;
    const int tx = (int)(lt % d.tiles_x), ty = (int)(lt / d.tiles_x);
    TileGeom g;
    g.i0 = (int64_t)tx << d.sx;
    g.j0 = (int64_t)ty << d.sy;
    const int TX = 1 << d.sx, TY = 1 << d.sy;
    g.w = d.nx - g.i0 < TX ? (int)(d.nx - g.i0) : TX;
    g.h = d.ny - g.j0 < TY ? (int)(d.ny - g.j0) : TY;
    return g;
}

// The tiles of the tile groups [g0, g0 + n_groups) (those of the simulations whose tiles run
// from bb.tile0 on).  first_slice / last_slice: whether the tiles start from +inf (else from
// the Z-map) and whether the first roughness pass runs; -1 takes both per simulation from the
// slice's rows [r0, r1) (histogram mode).  NT threads per block: tiles of more than 64 KiB of
// keys leave room for one block per compute unit, which then takes eight waves to keep enough
// bucket loads in flight.
template <int PREC, int NT>
__global__ __launch_bounds__(NT) void tile_reduce(const DevSim *__restrict__ sims, int n_sims,
                                                      const int64_t *__restrict__ group_base,
                                                      int64_t g0, int64_t n_groups, BinBuffers bb,
                                                      int first_slice, int last_slice, int64_t r0,
                                                      int64_t r1, TileStat1 *__restrict__ st1,
                                                      uint64_t *__restrict__ binned)
{
    using KT = KeyOf<PREC>;
    using Key = typename KT::T;
    extern __shared__ __align__(16) unsigned char smem[];
    Key *lds = reinterpret_cast<Key *>(smem);
    const FSM_GLOBAL Key *bkey = gptr(static_cast<const Key *>(bb.bkey));
    const FSM_GLOBAL uint16_t *bix = gptr(bb.bidx);
    const FSM_GLOBAL uint32_t *tile_lo = gptr(bb.tile_lo), *tile_hi = gptr(bb.tile_hi);
    const int tid = threadIdx.x;
    // entries past the capacity were never written (the planner sizes slices so that none
    // are dropped); the clamp keeps the reads inside the bucket arrays regardless
    const int64_t cap = bb.cap;
    auto clamp = [cap](uint32_t o) { return (int64_t)o < cap ? o : (uint32_t)cap; };
    // Bucket entries travel in units of E neighbours: E keys in one 16-byte load, their cells
    // in one 4- or 8-byte load.  A bucket [e0, e1) splits into whole units [u0, u1) and at most
    // E - 1 single entries at each end.  The first kDepth units per thread and the single
    // entries of a tile's bucket are loaded while the tile before it drains, and the bucket
    // bounds one tile further ahead still: a sparse tile's entries then arrive without two
    // dependent load latencies of their own.  Bucket entries are read once: non-temporal loads
    // keep them from displacing the Z-map, which the roughness passes read next.  Lanes past
    // the bucket's end load unit 0 and drop it.
    constexpr int E = KeyVec<Key>::n;
    using KU = typename KeyVec<Key>::T;
    typedef uint16_t CU __attribute__((ext_vector_type(E)));
    const FSM_GLOBAL KU *ukey = reinterpret_cast<const FSM_GLOBAL KU *>(bkey);
    const FSM_GLOBAL CU *uix = reinterpret_cast<const FSM_GLOBAL CU *>(bix);
    constexpr int kDepth = 8 / E;   // units in flight per thread (eight entries)
    KU ak[kDepth];
    CU ac[kDepth];
    Key ok = KT::inf;           // this thread's single entry, if any
    uint16_t oc = 0;
    bool has_one = false;
    uint32_t a0 = 0, a1 = 0;   // bucket of the tile whose first entries are in ak / ac / ok
    uint32_t n0 = 0, n1 = 0;   // bucket of the tile after it
    // This block's tiles: the tile groups g0 + blockIdx.x, + gridDim.x, ..., each group's
    // tiles in order.  A position is the group (inside the slice) and the tile inside its
    // simulation; ok: the position exists.
    struct Pos {
        int64_t gl, lt, lt_end;
        int si;
        bool ok;
    };
    auto group_pos = [&](int64_t gl) {
        Pos p;
        p.gl = gl;
        p.ok = gl < n_groups;
        p.si = 0;
        p.lt = p.lt_end = 0;
        if (p.ok) {
            const int64_t gg = g0 + gl;
            p.si = n_sims == 1 ? 0 : find_sim(group_base, n_sims, gg);
            const DevSim &d = sims[p.si];
            p.lt = (gg - d.tgroup_base) << d.tg_shift;
            const int64_t e = p.lt + ((int64_t)1 << d.tg_shift);
            p.lt_end = e < d.n_tiles ? e : d.n_tiles;
        }
        return p;
    };
    auto succ = [&](Pos p) {
        if (!p.ok) return p;
        if (++p.lt < p.lt_end) return p;
        return group_pos(p.gl + gridDim.x);
    };
    // slice-local tile index of a position
    auto local_tile = [&](const Pos &p) { return sims[p.si].tile_base + p.lt - bb.tile0; };
    auto bounds = [&](const Pos &p, uint32_t &o0, uint32_t &o1) {
        o0 = o1 = 0;
        if (p.ok) {
            const int64_t tl = local_tile(p);
            o0 = clamp(tile_lo[tl]);
            o1 = clamp(tile_hi[tl]);
        }
    };
    auto ahead = [&]() {
        const UnitSplit q = unit_split<E>(a0, a1);
#pragma unroll
        for (int v = 0; v < kDepth; ++v) {
            const uint32_t u = q.u0 + tid + v * NT;
            const uint32_t uu = u < q.u1 ? u : 0u;
            ak[v] = __builtin_nontemporal_load(&ukey[uu]);
            ac[v] = __builtin_nontemporal_load(&uix[uu]);
        }
        const uint32_t nh = q.hb - q.e0, nt = q.e1 - q.tb;
        has_one = (uint32_t)tid < nh + nt;
        if (has_one) {
            const uint32_t e = (uint32_t)tid < nh ? q.e0 + tid : q.tb + (tid - nh);
            ok = __builtin_nontemporal_load(&bkey[e]);
            oc = __builtin_nontemporal_load(&bix[e]);
        }
    };
    Pos pc = group_pos(blockIdx.x), pn = succ(pc);
    bounds(pc, a0, a1);
    bounds(pn, n0, n1);
    ahead();
    // first-pass partials of the current group; whether any of its tiles holds the feed /
    // pick profile's row / column
    Stat1Acc acc;
    bool grp_rows = false, grp_cols = false;
    while (pc.ok) {
        const DevSim d = sims[pc.si];
        const int64_t t = d.tile_base + pc.lt;
        const bool first = first_slice >= 0 ? first_slice != 0 : d.row_base >= r0;
        const bool last = last_slice >= 0 ? last_slice != 0 : d.row_base + d.n_rows <= r1;
        const TileGeom g = tile_geom(d, t);
        const int sx = d.sx, TX = 1 << sx, TC = TX << d.sy;
        FSM_GLOBAL Key *Z = gptr(static_cast<Key *>(d.zmap)) + g.j0 * d.nx + g.i0;
        // 16-byte vectors of cells along the tile's rows when every row of the map starts on
        // a 16-byte boundary and the tile's width is a whole number of vectors (a vector then
        // lies wholly inside or wholly outside the grid); single cells otherwise
        constexpr int V = KeyVec<Key>::n;
        using Vec = typename KeyVec<Key>::T;
        const bool vec = (((uintptr_t)d.zmap | (uintptr_t)(d.nx * (int64_t)sizeof(Key))) & 15) == 0 &&
                         (g.w & (V - 1)) == 0;
        if (vec) {
            for (int l = tid * V; l < TC; l += NT * V) {
                const int li = l & (TX - 1), lj = l >> sx;
                Vec v = (Vec)KT::inf;
                if (!first && li < g.w && lj < g.h) {
                    v = *reinterpret_cast<const FSM_GLOBAL Vec *>(Z + (int64_t)lj * d.nx + li);
#pragma unroll
                    for (int c = 0; c < V; ++c) v[c] = KT::enc(v[c]);
                }
                *reinterpret_cast<Vec *>(lds + l) = v;
            }
        } else {
            for (int l = tid; l < TC; l += NT) {
                const int li = l & (TX - 1), lj = l >> sx;
                Key v = KT::inf;
                if (!first && li < g.w && lj < g.h) v = KT::enc(Z[(int64_t)lj * d.nx + li]);
                lds[l] = v;
            }
        }
        __syncthreads();
        const uint32_t e0 = a0, e1 = a1;
        const UnitSplit q = unit_split<E>(e0, e1);
        if (has_one) __hip_atomic_fetch_min(&lds[oc], ok, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
        for (int v = 0; v < kDepth; ++v)
            if (q.u0 + tid + v * NT < q.u1) {
#pragma unroll
                for (int c = 0; c < E; ++c)
                    __hip_atomic_fetch_min(&lds[ac[v][c]], ak[v][c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        uint32_t u = q.u0 + tid + kDepth * NT;
        for (; u + (kDepth - 1) * NT < q.u1; u += kDepth * NT) {
            KU k4[kDepth];
            CU c4[kDepth];
#pragma unroll
            for (int v = 0; v < kDepth; ++v) {
                k4[v] = __builtin_nontemporal_load(&ukey[u + v * NT]);
                c4[v] = __builtin_nontemporal_load(&uix[u + v * NT]);
            }
#pragma unroll
            for (int v = 0; v < kDepth; ++v)
#pragma unroll
                for (int c = 0; c < E; ++c)
                    __hip_atomic_fetch_min(&lds[c4[v][c]], k4[v][c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        for (; u < q.u1; u += NT) {
            const KU k1 = __builtin_nontemporal_load(&ukey[u]);
            const CU c1 = __builtin_nontemporal_load(&uix[u]);
#pragma unroll
            for (int c = 0; c < E; ++c)
                __hip_atomic_fetch_min(&lds[c1[c]], k1[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (tid == 0 && e1 > e0) atomicAdd((unsigned long long *)(binned + d.sim), (unsigned long long)(e1 - e0));
        __syncthreads();
        // the next tile's first entries travel while this one drains
        const Pos pn2 = succ(pn);
        a0 = n0;
        a1 = n1;
        bounds(pn2, n0, n1);
        ahead();
        const int64_t rj = d.ny / 2 - g.j0, ci = d.nx / 2 - g.i0;
        grp_rows |= rj >= 0 && rj < g.h;
        grp_cols |= ci >= 0 && ci < g.w;
        if (vec) {
            for (int l = tid * V; l < TC; l += NT * V) {
                const int li = l & (TX - 1), lj = l >> sx;
                if (li < g.w && lj < g.h) {
                    Vec v = *reinterpret_cast<const Vec *>(lds + l);
#pragma unroll
                    for (int c = 0; c < V; ++c) v[c] = KT::enc(v[c]);
                    *reinterpret_cast<FSM_GLOBAL Vec *>(Z + (int64_t)lj * d.nx + li) = v;
                    if (last) {
                        double h[V];
#pragma unroll
                        for (int c = 0; c < V; ++c) h[c] = KT::height(v[c]);
                        const int64_t at = ci - li;
                        acc.add_vec<V>(h, lj == rj, at >= 0 && at < V ? (int)at : -1);
                    }
                }
            }
        } else {
            for (int l = tid; l < TC; l += NT) {
                const int li = l & (TX - 1), lj = l >> sx;
                if (li < g.w && lj < g.h) {
                    const Key k = KT::enc(lds[l]);
                    Z[(int64_t)lj * d.nx + li] = k;
                    if (last) acc.add(KT::height(k), lj == rj, li == ci);
                }
            }
        }
        if (last) {
            // one block reduction per group: its partials go to the group's last tile, the
            // other tiles of the group get empty ones
            if (pc.lt + 1 == pc.lt_end) {
                const TileStat1 s = acc.reduce<NT / 64>(grp_rows, grp_cols, true);
                if (tid == 0) st1[t] = s;
                acc = Stat1Acc();
                grp_rows = grp_cols = false;
            } else if (tid == 0) {
                st1[t] = Stat1Acc().partial();
            }
        }
        __syncthreads();
        pc = pn;
        pn = pn2;
    }
}

// ---- tiled roughness ---------------------------------------------------------------------------

// First pass over tiles of finished Z-maps: optional decoding of scatter keys (only negative
// heights change bits, so only those are written back) and the tile partial sums.
template <int PREC>
__global__ __launch_bounds__(kBlock) void tile_stats1(const DevSim *__restrict__ sims, int n_sims,
                                                      const int64_t *__restrict__ tile_base,
                                                      int64_t n_tiles, int decode, TileStat1 *st1)
{
    using KT = KeyOf<PREC>;
    using Key = typename KT::T;
    const int tid = threadIdx.x;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int si = n_sims == 1 ? 0 : find_sim(tile_base, n_sims, t);
        const DevSim d = sims[si];
        const TileGeom g = tile_geom(d, t);
        const int TX = 1 << d.sx, TC = TX << d.sy;
        FSM_GLOBAL Key *Z = gptr(static_cast<Key *>(d.zmap)) + g.j0 * d.nx + g.i0;
        const int64_t rj = d.ny / 2 - g.j0, ci = d.nx / 2 - g.i0;
        Stat1Acc acc;
        for (int l = tid; l < TC; l += kBlock) {
            const int li = l & (TX - 1), lj = l >> d.sx;
            if (li < g.w && lj < g.h) {
                Key k = Z[(int64_t)lj * d.nx + li];
                if (decode && k < 0) {
                    k = KT::enc(k);
                    Z[(int64_t)lj * d.nx + li] = k;
                }
                acc.add(KT::height(k), lj == rj, li == ci);
            }
        }
        const TileStat1 s = acc.reduce(rj >= 0 && rj < g.h, ci >= 0 && ci < g.w, true);
        if (tid == 0) st1[t] = s;
    }
}

constexpr int kFinalDepth = 8;   // tile partials in flight per thread of the final combines

// One block per simulation: combine its tile groups' first-pass partials in a fixed order.
__global__ __launch_bounds__(kBlock) void rough_final1(const DevSim *__restrict__ sims,
                                                       const TileStat1 *__restrict__ st1,
                                                       RoughState *state)
{
    const DevSim d = sims[blockIdx.x];
    Stat1Acc a;
    auto add = [&a](const TileStat1 &s) {
        a.sum += s.sum;
        a.mn = fmin(a.mn, s.mn);
        a.mx = fmax(a.mx, s.mx);
        a.row_sum += s.row_sum;
        a.col_sum += s.col_sum;
        a.n += s.n;
        a.row_n += s.row_n;
        a.col_n += s.col_n;
    };
    // the partials of the tile groups (each at its group's last tile; the other tiles' are
    // empty, and so are all of a scatter-strategy pass's but the ones read here when the
    // groups are single tiles), each thread's in order with kFinalDepth in flight
    const TileStat1 *p = st1 + d.tile_base;
    const int sh = d.tg_shift;
    auto at = [&](int64_t g) {
        const int64_t e = (g + 1) << sh;
        return p[(e < d.n_tiles ? e : d.n_tiles) - 1];
    };
    int64_t k = threadIdx.x;
    for (; k + (kFinalDepth - 1) * kBlock < d.n_tgroups; k += kFinalDepth * kBlock) {
        TileStat1 s[kFinalDepth];
#pragma unroll
        for (int v = 0; v < kFinalDepth; ++v) s[v] = at(k + v * kBlock);
#pragma unroll
        for (int v = 0; v < kFinalDepth; ++v) add(s[v]);
    }
    for (; k < d.n_tgroups; k += kBlock) add(at(k));
    const TileStat1 r = a.reduce();
    if (threadIdx.x == 0) {
        RoughState st;
        st.n = r.n;
        st.mean = r.n ? r.sum / (double)r.n : NAN;
        st.mn = r.mn;
        st.mx = r.mx;
        st.n_row = r.row_n;
        st.row_mean = r.row_n ? r.row_sum / (double)r.row_n : NAN;
        st.n_col = r.col_n;
        st.col_mean = r.col_n ? r.col_sum / (double)r.col_n : NAN;
        state[d.sim] = st;
    }
}

struct Stat2Acc {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, row_abs = 0.0, col_abs = 0.0;
    __device__ TileStat2 reduce()
    {
        __shared__ double bd[4];
        TileStat2 t;
        t.s1 = block_sum(s1, bd);
        t.s2 = block_sum(s2, bd);
        t.s3 = block_sum(s3, bd);
        t.s4 = block_sum(s4, bd);
        t.row_abs = block_sum(row_abs, bd);
        t.col_abs = block_sum(col_abs, bd);
        return t;
    }
};

// Second pass: central moments about each simulation's mean, and the profile deviations.  One
// block per tile, its threads over consecutive cells of the tile's rows with kRows2 loads in
// flight each (16-byte vectors of cells when the map's rows allow it, as in tile_reduce); the
// waves' butterfly sums are combined left to right after one barrier.
constexpr int kRows2 = 8;
struct Moments {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, row_abs = 0.0, col_abs = 0.0;
    // V neighbouring cells of one map row, +inf (not cut) counting nowhere; their terms are
    // summed among themselves first, which shortens the dependency chains
    template <int V>
    __device__ void add(const double (&v)[V], const RoughState &st, bool row_hit, int col_at)
    {
        double a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, ra = 0.0;
#pragma unroll
        for (int c = 0; c < V; ++c) {
            const bool h = v[c] < INFINITY;
            const double dv = h ? v[c] - st.mean : 0.0;
            const double d2 = dv * dv;
            a1 += fabs(dv);
            a2 += d2;
            a3 += d2 * dv;
            a4 += d2 * d2;
            if (row_hit && h) ra += fabs(v[c] - st.row_mean);
            if (c == col_at && h) col_abs += fabs(v[c] - st.col_mean);
        }
        s1 += a1;
        s2 += a2;
        s3 += a3;
        s4 += a4;
        row_abs += ra;
    }
};

template <int PREC>
__global__ __launch_bounds__(kBlock) void tile_stats2(const DevSim *__restrict__ sims, int n_sims,
                                                      const int64_t *__restrict__ tile_base,
                                                      int64_t n_tiles, const RoughState *__restrict__ state,
                                                      TileStat2 *st2)
{
    using KT = KeyOf<PREC>;
    using Key = typename KT::T;
    constexpr int V = KeyVec<Key>::n;
    using Vec = typename KeyVec<Key>::T;
    __shared__ double part[6][kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int si = n_sims == 1 ? 0 : find_sim(tile_base, n_sims, t);
        const DevSim &d = sims[si];
        const RoughState st = state[d.sim];
        const TileGeom g = tile_geom(d, t);
        const int sx = d.sx, TX = 1 << sx, TC = TX << d.sy;
        const int64_t nx = d.nx;
        const FSM_GLOBAL Key *Z = gptr(static_cast<const Key *>(d.zmap)) + g.j0 * nx + g.i0;
        const int64_t rj = d.ny / 2 - g.j0, ci = d.nx / 2 - g.i0;
        Moments m;
        const bool vec = (((uintptr_t)d.zmap | (uintptr_t)(nx * (int64_t)sizeof(Key))) & 15) == 0 &&
                         (g.w & (V - 1)) == 0;
        if (vec) {
            for (int l0 = tid * V; l0 < TC; l0 += kRows2 * kBlock * V) {
                // every load is issued (vectors outside the tile read its first one) so that
                // all kRows2 are in flight together; their values are masked afterwards
                Vec k[kRows2];
#pragma unroll
                for (int u = 0; u < kRows2; ++u) {
                    const int l = l0 + u * kBlock * V, li = l & (TX - 1), lj = l >> sx;
                    const bool in = l < TC && li < g.w && lj < g.h;
                    k[u] = *reinterpret_cast<const FSM_GLOBAL Vec *>(Z + (in ? (int64_t)lj * nx + li : 0));
                }
#pragma unroll
                for (int u = 0; u < kRows2; ++u) {
                    const int l = l0 + u * kBlock * V, li = l & (TX - 1), lj = l >> sx;
                    const bool in = l < TC && li < g.w && lj < g.h;
                    double v[V];
#pragma unroll
                    for (int c = 0; c < V; ++c) v[c] = in ? KT::height(k[u][c]) : INFINITY;
                    const int64_t at = ci - li;
                    m.add<V>(v, st, lj == rj, at >= 0 && at < V ? (int)at : -1);
                }
            }
        } else {
            for (int l0 = tid; l0 < TC; l0 += kRows2 * kBlock) {
                Key k[kRows2];
#pragma unroll
                for (int u = 0; u < kRows2; ++u) {
                    const int l = l0 + u * kBlock, li = l & (TX - 1), lj = l >> sx;
                    const bool in = l < TC && li < g.w && lj < g.h;
                    k[u] = Z[in ? (int64_t)lj * nx + li : 0];
                }
#pragma unroll
                for (int u = 0; u < kRows2; ++u) {
                    const int l = l0 + u * kBlock, li = l & (TX - 1), lj = l >> sx;
                    const bool in = l < TC && li < g.w && lj < g.h;
                    const double v[1] = {in ? KT::height(k[u]) : INFINITY};
                    m.add<1>(v, st, lj == rj, li == ci ? 0 : -1);
                }
            }
        }
        double s1 = m.s1, s2 = m.s2, s3 = m.s3, s4 = m.s4, row_abs = m.row_abs, col_abs = m.col_abs;
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        s3 = wave_sum(s3);
        s4 = wave_sum(s4);
        // the profile terms are zero in every thread of a tile off the profile lines
        if (rj >= 0 && rj < g.h) row_abs = wave_sum(row_abs);
        if (ci >= 0 && ci < g.w) col_abs = wave_sum(col_abs);
        if (lane == 0) {
            part[0][wv] = s1;
            part[1][wv] = s2;
            part[2][wv] = s3;
            part[3][wv] = s4;
            part[4][wv] = row_abs;
            part[5][wv] = col_abs;
        }
        __syncthreads();
        if (tid == 0) {
            TileStat2 r;
            r.s1 = (part[0][0] + part[0][1]) + (part[0][2] + part[0][3]);
            r.s2 = (part[1][0] + part[1][1]) + (part[1][2] + part[1][3]);
            r.s3 = (part[2][0] + part[2][1]) + (part[2][2] + part[2][3]);
            r.s4 = (part[3][0] + part[3][1]) + (part[3][2] + part[3][3]);
            r.row_abs = (part[4][0] + part[4][1]) + (part[4][2] + part[4][3]);
            r.col_abs = (part[5][0] + part[5][1]) + (part[5][2] + part[5][3]);
            st2[t] = r;
        }
        __syncthreads();
    }
}

// One block per simulation: combine the second-pass partials and write the result record.
__global__ __launch_bounds__(kBlock) void rough_final2(const DevSim *__restrict__ sims,
                                                       const TileStat2 *__restrict__ st2,
                                                       const RoughState *__restrict__ state,
                                                       const uint64_t *__restrict__ binned,
                                                       const int64_t *__restrict__ evals,
                                                       fsm_rough *out)
{
    const DevSim d = sims[blockIdx.x];
    Stat2Acc a;
    auto add = [&a](const TileStat2 &s) {
        a.s1 += s.s1;
        a.s2 += s.s2;
        a.s3 += s.s3;
        a.s4 += s.s4;
        a.row_abs += s.row_abs;
        a.col_abs += s.col_abs;
    };
    const TileStat2 *p = st2 + d.tile_base;
    constexpr int D = 2 * kFinalDepth;
    int64_t k = threadIdx.x;
    for (; k + (D - 1) * kBlock < d.n_tiles; k += D * kBlock) {
        TileStat2 s[D];
#pragma unroll
        for (int v = 0; v < D; ++v) s[v] = p[k + v * kBlock];
#pragma unroll
        for (int v = 0; v < D; ++v) add(s[v]);
    }
    for (; k < d.n_tiles; k += kBlock) add(p[k]);
    const TileStat2 r = a.reduce();
    // the per-row near-boundary counts of the histogram mode
    uint64_t near_rows = 0;
    if (d.near_rows) {
        __shared__ uint64_t nb[kWaves];
        for (int64_t k = threadIdx.x; k < d.n_rows; k += kBlock) near_rows += d.near_rows[d.row_base + k];
        near_rows = block_sum(near_rows, nb);
    }
    if (threadIdx.x == 0) {
        const RoughState st = state[d.sim];
        fsm_rough o;
        const int64_t n = st.n;
        const double dn = (double)n;
        o.n_hit = n;
        o.n_evals = evals ? evals[d.sim] : 0;
        o.n_binned = binned ? (int64_t)binned[d.sim] : 0;
        o.n_feed = st.n_row;
        o.n_pick = st.n_col;
        o.flags = 0;
        o.reserved = 0;
        o.mean = st.mean;
        o.pos_err = d.pos_err;
        o.n_near = (d.near ? (int64_t)*d.near : 0) + (int64_t)near_rows;
        if (n == 0) {
            o.Sa = o.Sq = o.Sp = o.Sv = o.Sz = o.Ssk = o.Sku = NAN;
            o.flags |= FSM_FLAG_NO_HIT;
        } else {
            o.Sa = r.s1 / dn;
            o.Sq = sqrt(r.s2 / dn);
            o.Sp = st.mx - st.mean;
            o.Sv = st.mean - st.mn;
            o.Sz = o.Sp + o.Sv;
            if (o.Sq > 0.0) {
                o.Ssk = (r.s3 / dn) / (o.Sq * o.Sq * o.Sq);
                o.Sku = (r.s4 / dn) / (o.Sq * o.Sq * o.Sq * o.Sq);
            } else {
                o.Ssk = o.Sku = NAN;
                o.flags |= FSM_FLAG_SQ_ZERO;
            }
        }
        if ((double)n < 0.99 * (double)d.nx * (double)d.ny) o.flags |= FSM_FLAG_LOW_COVERAGE;
        o.Ra_feed = st.n_row ? r.row_abs / (double)st.n_row : NAN;
        o.Ra_pick = st.n_col ? r.col_abs / (double)st.n_col : NAN;
        out[d.sim] = o;
    }
}

}  // namespace

// ---- launch wrappers ---------------------------------------------------------------------------

int launch_fill(const DevSim *d_sims, int n_sims, int64_t max_cells, int precision, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int blocks = stream_blocks(max_cells, (int64_t)kBlock * 8, 8192);
    if (precision == FSM_F64)
        hipLaunchKernelGGL(fill_maps<int64_t>, dim3(blocks), dim3(kBlock), 0, s, d_sims, n_sims, (int64_t)kInf64);
    else
        hipLaunchKernelGGL(fill_maps<int32_t>, dim3(blocks), dim3(kBlock), 0, s, d_sims, n_sims, (int32_t)kInf32);
    return (int)hipGetLastError();
}

int launch_scatter(const DevSim *d_sims, int n_sims, const int64_t *d_item_base, int64_t n_items,
                   int precision, uint64_t *d_binned, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int blocks = (int)(n_items < kMaxGrid ? n_items : kMaxGrid);
    if (blocks <= 0) return 0;
    if (precision == FSM_F64)
        hipLaunchKernelGGL(scatter<FSM_F64>, dim3(blocks), dim3(kBlock), 0, s, d_sims, n_sims, d_item_base, n_items, d_binned);
    else
        hipLaunchKernelGGL(scatter<FSM_F32>, dim3(blocks), dim3(kBlock), 0, s, d_sims, n_sims, d_item_base, n_items, d_binned);
    return (int)hipGetLastError();
}

namespace {

void stage(const StageEvents *marks, int k, hipStream_t s)
{
    if (marks) (void)hipEventRecord(static_cast<hipEvent_t>(marks->ev[k]), s);
}

// Exclusive scan of counts[0, n) into offsets and cursors.
void launch_scan(int64_t n_tiles, const BinBuffers &bb, hipStream_t s)
{
    if (n_tiles <= kScanSeg) {
        // one segment: one launch
        hipLaunchKernelGGL(scan_single, dim3(1), dim3(kBlock), 0, s, (const uint32_t *)bb.counts, n_tiles, bb.offsets, bb.cursor);
        return;
    }
    const int nb = (int)((n_tiles + kScanSeg - 1) / kScanSeg);
    hipLaunchKernelGGL(scan_reduce, dim3(nb), dim3(kBlock), 0, s, (const uint32_t *)bb.counts, n_tiles, bb.bsum);
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(kBlock), 0, s, bb.bsum, nb, bb.offsets, n_tiles);
    hipLaunchKernelGGL(scan_apply, dim3(nb), dim3(kBlock), 0, s, (const uint32_t *)bb.counts, n_tiles, (const uint32_t *)bb.bsum, bb.offsets, bb.cursor);
}

template <int PREC>
void binned_slice(const DevSim *d_sims, int n_sims, const int64_t *d_bitem_base,
                  int64_t n_tiles, const int64_t *d_gbase, int64_t g0,
                  int64_t n_groups, int64_t item_begin, int64_t n_items, const BinBuffers &bb,
                  bool first_slice, bool last_slice, int sx, int sy, TileStat1 *st1,
                  uint64_t *d_binned, hipStream_t s, const StageEvents *marks)
{
    const int ib = (int)(n_items < kMaxGrid ? n_items : kMaxGrid);
    const int tb = (int)(n_groups < kMaxGrid ? n_groups : kMaxGrid);
    const size_t lds = sizeof(typename KeyOf<PREC>::T) << (sx + sy);
    stage(marks, 0, s);
    hipLaunchKernelGGL(zero_u32, dim3(stream_blocks(n_tiles, kBlock, 4096)), dim3(kBlock), 0, s, bb.counts, n_tiles);
    if (ib > 0)
        hipLaunchKernelGGL((bin_points<PREC, false>), dim3(ib), dim3(kBlock), 0, s, d_sims, n_sims, d_bitem_base, item_begin, n_items, bb);
    stage(marks, 1, s);
    launch_scan(n_tiles, bb, s);
    stage(marks, 2, s);
    if (ib > 0)
        hipLaunchKernelGGL((bin_points<PREC, true>), dim3(ib), dim3(kBlock), 0, s, d_sims, n_sims, d_bitem_base, item_begin, n_items, bb);
    stage(marks, 3, s);
    if (tb > 0 && lds > kTileLdsSmall)
        hipLaunchKernelGGL((tile_reduce<PREC, 2 * kBlock>), dim3(tb), dim3(2 * kBlock), lds, s, d_sims, n_sims, d_gbase, g0, n_groups, bb, first_slice ? 1 : 0, last_slice ? 1 : 0, (int64_t)0, (int64_t)0, st1, d_binned);
    else if (tb > 0)
        hipLaunchKernelGGL((tile_reduce<PREC, kBlock>), dim3(tb), dim3(kBlock), lds, s, d_sims, n_sims, d_gbase, g0, n_groups, bb, first_slice ? 1 : 0, last_slice ? 1 : 0, (int64_t)0, (int64_t)0, st1, d_binned);
    stage(marks, 4, s);
}

template <int PREC>
void hist_slice(const DevSim *d_sims, int n_sims, const int64_t *d_row_base,
                const int64_t *d_hbase, int64_t n_htiles, const int64_t *d_gbase, int64_t g0,
                int64_t n_groups,
                int64_t row_begin, int64_t row_end, const BinBuffers &bb, int sx, int sy,
                TileStat1 *st1, uint64_t *d_binned, hipStream_t s, const StageEvents *marks)
{
    const int64_t nr = row_end - row_begin;
    const int rb = (int)(nr < kMaxGrid ? nr : kMaxGrid);
    const size_t hist_lds = sizeof(uint32_t) * (size_t)(bb.max_tiles > 0 ? bb.max_tiles : 1);
    const int64_t n_chunks = (nr + bb.row_chunk - 1) / bb.row_chunk;
    const int cb = stream_blocks(n_chunks * n_htiles, kBlock, 16384);
    const int tb1 = stream_blocks(n_htiles, kBlock, 16384);
    const int hb = (int)(n_htiles < kMaxGrid ? n_htiles : kMaxGrid);
    const int tb = (int)(n_groups < kMaxGrid ? n_groups : kMaxGrid);
    const size_t lds = sizeof(typename KeyOf<PREC>::T) << (sx + sy);
    const bool super = bb.skey != nullptr;
    stage(marks, 0, s);
    if (rb > 0)
        hipLaunchKernelGGL(hist_count<PREC>, dim3(rb), dim3(kBlock), hist_lds, s, d_sims, n_sims, d_row_base, row_begin, nr, bb);
    stage(marks, 1, s);
    if (n_chunks > 0) {
        hipLaunchKernelGGL(hist_colsum, dim3(cb), dim3(kBlock), 0, s, d_sims, n_sims, d_hbase, n_htiles, row_begin, row_end, n_chunks, bb);
        hipLaunchKernelGGL(hist_chunkscan, dim3(tb1), dim3(kBlock), 0, s, n_htiles, n_chunks, bb);
        hipLaunchKernelGGL(hist_apply, dim3(cb), dim3(kBlock), 0, s, d_sims, n_sims, d_hbase, n_htiles, row_begin, row_end, n_chunks, bb);
    } else {
        hipLaunchKernelGGL(zero_u32, dim3(tb1), dim3(kBlock), 0, s, bb.counts, n_htiles);
    }
    launch_scan(n_htiles, bb, s);
    stage(marks, 2, s);
    if (rb > 0) {
        if (super)
            hipLaunchKernelGGL((hist_write<PREC, true>), dim3(rb), dim3(kBlock), hist_lds, s, d_sims, n_sims, d_row_base, row_begin, nr, bb);
        else
            hipLaunchKernelGGL((hist_write<PREC, false>), dim3(rb), dim3(kBlock), hist_lds, s, d_sims, n_sims, d_row_base, row_begin, nr, bb);
    }
    if (super && hb > 0)
        hipLaunchKernelGGL(split_super<PREC>, dim3(hb), dim3(kBlock), 0, s, d_sims, n_sims, d_hbase, n_htiles, bb);
    stage(marks, 3, s);
    if (tb > 0 && lds > kTileLdsSmall)
        hipLaunchKernelGGL((tile_reduce<PREC, 2 * kBlock>), dim3(tb), dim3(2 * kBlock), lds, s, d_sims, n_sims, d_gbase, g0, n_groups, bb, -1, -1, row_begin, row_end, st1, d_binned);
    else if (tb > 0)
        hipLaunchKernelGGL((tile_reduce<PREC, kBlock>), dim3(tb), dim3(kBlock), lds, s, d_sims, n_sims, d_gbase, g0, n_groups, bb, -1, -1, row_begin, row_end, st1, d_binned);
    stage(marks, 4, s);
}

}  // namespace

int launch_binned_slice(const DevSim *d_sims, int n_sims, const int64_t *d_bitem_base,
                        int64_t n_tiles, const int64_t *d_gbase,
                        int64_t g0, int64_t n_groups, int64_t item_begin, int64_t n_items,
                        const BinBuffers &bb, bool first_slice, bool last_slice, int precision,
                        int sx, int sy, TileStat1 *st1, uint64_t *d_binned, void *stream,
                        const StageEvents *marks)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == FSM_F64)
        binned_slice<FSM_F64>(d_sims, n_sims, d_bitem_base, n_tiles, d_gbase, g0, n_groups, item_begin, n_items, bb, first_slice, last_slice, sx, sy, st1, d_binned, s, marks);
    else
        binned_slice<FSM_F32>(d_sims, n_sims, d_bitem_base, n_tiles, d_gbase, g0, n_groups, item_begin, n_items, bb, first_slice, last_slice, sx, sy, st1, d_binned, s, marks);
    return (int)hipGetLastError();
}

int launch_hist_slice(const DevSim *d_sims, int n_sims, const int64_t *d_row_base,
                      const int64_t *d_hbase, int64_t n_htiles, const int64_t *d_gbase,
                      int64_t g0, int64_t n_groups,
                      int64_t row_begin, int64_t row_end, const BinBuffers &bb, int precision,
                      int sx, int sy, TileStat1 *st1, uint64_t *d_binned, void *stream,
                      const StageEvents *marks)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == FSM_F64)
        hist_slice<FSM_F64>(d_sims, n_sims, d_row_base, d_hbase, n_htiles, d_gbase, g0, n_groups, row_begin, row_end, bb, sx, sy, st1, d_binned, s, marks);
    else
        hist_slice<FSM_F32>(d_sims, n_sims, d_row_base, d_hbase, n_htiles, d_gbase, g0, n_groups, row_begin, row_end, bb, sx, sy, st1, d_binned, s, marks);
    return (int)hipGetLastError();
}


int launch_trajectory(const DevSim *d_sim, int64_t n_items, int precision, void *traj,
                      int32_t *index, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int ib = (int)(n_items < kMaxGrid ? n_items : kMaxGrid);
    if (ib > 0) {
        if (precision == FSM_F64)
            hipLaunchKernelGGL(trajectory<FSM_F64>, dim3(ib), dim3(kBlock), 0, s, d_sim, n_items, traj, index);
        else
            hipLaunchKernelGGL(trajectory<FSM_F32>, dim3(ib), dim3(kBlock), 0, s, d_sim, n_items, traj, index);
    }
    return (int)hipGetLastError();
}

int launch_rough(const DevSim *d_sims, int n_sims, const int64_t *d_tile_base, int64_t n_tiles,
                 int precision, int, int, bool with_pass1, bool decode, TileStat1 *st1,
                 TileStat2 *st2, RoughState *state, const uint64_t *d_binned,
                 const int64_t *d_evals, fsm_rough *d_out, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int tb = (int)(n_tiles < kMaxGrid ? n_tiles : kMaxGrid);
    if (with_pass1) {
        if (precision == FSM_F64)
            hipLaunchKernelGGL(tile_stats1<FSM_F64>, dim3(tb), dim3(kBlock), 0, s, d_sims, n_sims, d_tile_base, n_tiles, decode ? 1 : 0, st1);
        else
            hipLaunchKernelGGL(tile_stats1<FSM_F32>, dim3(tb), dim3(kBlock), 0, s, d_sims, n_sims, d_tile_base, n_tiles, decode ? 1 : 0, st1);
    }
    hipLaunchKernelGGL(rough_final1, dim3(n_sims), dim3(kBlock), 0, s, d_sims, (const TileStat1 *)st1, state);
    if (precision == FSM_F64)
        hipLaunchKernelGGL(tile_stats2<FSM_F64>, dim3(tb), dim3(kBlock), 0, s, d_sims, n_sims, d_tile_base, n_tiles, (const RoughState *)state, st2);
    else
        hipLaunchKernelGGL(tile_stats2<FSM_F32>, dim3(tb), dim3(kBlock), 0, s, d_sims, n_sims, d_tile_base, n_tiles, (const RoughState *)state, st2);
    hipLaunchKernelGGL(rough_final2, dim3(n_sims), dim3(kBlock), 0, s, d_sims, (const TileStat2 *)st2, (const RoughState *)state, d_binned, d_evals, d_out);
    return (int)hipGetLastError();
}

}  // namespace fsm
