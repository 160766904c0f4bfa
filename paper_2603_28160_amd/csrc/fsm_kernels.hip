// fsm_kernels.hip -- gfx950 kernels of libfsm.
//
//   fill      : Z-map <- +inf (the empty-cell value) with 16-byte stores.
//   scatter   : the hot loop of the method (Sec. 2.3, Sec. 3.2 "surface computation"): every
//               (pass, step, tooth, edge point) is turned into the workpiece frame (Eq. (3)-(5)
//               plus tilt) on the fly, binned into its half-open sampling boundary (Eq. (7)) and
//               min-reduced into the Z-map with an integer atomic min on an order-preserving
//               encoding of the height.  One block owns one (pass, step chunk, tooth) item.
//   rough     : two passes over the Z-map (count/sum/min/max, then central moments) with
//               wave64 shuffles and a fixed-order combine; a one-block finalize computes the
//               ISO 25178-2 amplitude parameters and the two profile Ra values.
//
// Double precision: only +, -, * run on the device (no contraction: -ffp-contract=off), in
// the order the host planner documents, so binning decisions equal those of the plain
// definition bit for bit.  Single precision: rotation and tilt in float with fused
// multiply-adds; the tool-centre offset and the binning stay in double.
#include <hip/hip_runtime.h>

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

constexpr int64_t kInf64 = 0x7FF0000000000000LL;   // bits of +inf (double)
constexpr int32_t kInf32 = 0x7F800000;             // bits of +inf (float)

// Order-preserving map from IEEE heights to signed integers: non-negative values keep their
// bits, negative ones get every bit but the sign flipped.  The map is its own inverse.
__device__ __forceinline__ int64_t enc64(int64_t b) { return b >= 0 ? b : (b ^ 0x7FFFFFFFFFFFFFFFLL); }
__device__ __forceinline__ int32_t enc32(int32_t b) { return b >= 0 ? b : (b ^ 0x7FFFFFFF); }

// Block b of a launch runs on XCD (b mod 8).  Give every XCD a contiguous range of items so
// that the items sharing one XCD's L2 are neighbours along the tool path.
__device__ __forceinline__ int64_t xcd_item(int64_t b, int64_t G)
{
    const int64_t g8 = G >> 3;
    if (b >= (g8 << 3)) return b;
    return (b & 7) * g8 + (b >> 3);
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

// Block-wide reductions of kBlock (= 4 waves) threads; the result is valid in every thread.
// `buf` must hold 4 values.  Fixed order: lanes by butterfly, waves 0..3 left to right.
template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, T *buf, Op op)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) buf[w] = v;
    __syncthreads();
    return op(op(buf[0], buf[1]), op(buf[2], buf[3]));
}

// ---- fill ------------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void fill64(int64_t *z, int64_t n)
{
    const int64_t n2 = n >> 1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    longlong2 v = {kInf64, kInf64};
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n2; k += stride)
        reinterpret_cast<longlong2 *>(z)[k] = v;
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) z[n - 1] = kInf64;
}

__global__ __launch_bounds__(kBlock) void fill32(int32_t *z, int64_t n)
{
    const int64_t n4 = n >> 2;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int4 v = {kInf32, kInf32, kInf32, kInf32};
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n4; k += stride)
        reinterpret_cast<int4 *>(z)[k] = v;
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) z[(n4 << 2) + threadIdx.x] = kInf32;
}

// ---- scatter ---------------------------------------------------------------------------------

// Index of the simulation that owns global work item `item` (item_base is ascending, with
// item_base[0] == 0).
__device__ __forceinline__ int find_sim(const int64_t *__restrict__ base, int n, int64_t item)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void scatter(const DevSim *__restrict__ sims, int n_sims,
                                                  const int64_t *__restrict__ item_base,
                                                  int64_t n_items, uint64_t *__restrict__ binned)
{
    __shared__ uint32_t red[4];
    uint32_t cnt = 0;
    const int tid = threadIdx.x;
    for (int64_t b = blockIdx.x; b < n_items; b += gridDim.x) {
        // items of one round of the grid, spread over the XCDs in contiguous ranges
        const int64_t round0 = b - blockIdx.x;
        const int64_t rn = n_items - round0 < (int64_t)gridDim.x ? n_items - round0 : (int64_t)gridDim.x;
        const int64_t item = round0 + xcd_item(b - round0, rn);
        const int si = n_sims == 1 ? 0 : find_sim(item_base, n_sims, item);
        const DevSim d = sims[si];
        int64_t local = item - d.item_base;
        const int K = (int)(local % d.z_n);
        local /= d.z_n;
        const int chunk = (int)(local % d.n_chunks);
        const int q = (int)(local / d.n_chunks);

        const int ppi = d.ppi, spi = d.spi;
        const int lane_p = tid % ppi, lane_s = tid / ppi;
        if (lane_s >= spi) continue;
        const int s0 = chunk * d.chunk;
        const int s1 = s0 + d.chunk < d.n_steps ? s0 + d.chunk : d.n_steps;
        const double yq = d.y_first + (double)q * d.a_e;
        const int S = d.S;
        const double x_lo = d.x_lo, y_lo = d.y_lo, inv = d.inv_dd;
        const double nxd = d.nx_d, nyd = d.ny_d;
        const int64_t nx = d.nx;
        const FSM_GLOBAL double *__restrict__ xc = gptr(d.xc);

        for (int p = lane_p; p < d.N; p += ppi) {
            int s = s0 + lane_s;
            int m = s % S;
            if (PREC == FSM_F64) {
                const FSM_GLOBAL double *__restrict__ cs = gptr(d.cs + (size_t)K * S * 2);
                const FSM_GLOBAL double *pt = gptr(d.pT + ((size_t)K * d.N + p) * 3);
                const double xT = pt[0], yT = pt[1], zT = pt[2];
                FSM_GLOBAL int64_t *__restrict__ zk = gptr(static_cast<int64_t *>(d.zmap));
                for (; s < s1; s += spi) {
                    const double ca = cs[2 * m], sa = cs[2 * m + 1];
                    // Eq. (3): [[c, s], [-s, c]] applied to the tool-frame point
                    double xs = ca * xT + sa * yT;
                    double ys = ca * yT - sa * xT;
                    double zs = zT;
                    if (d.tilt_lead) {
                        const double x1 = d.tl_c * xs + d.tl_s * zs;
                        zs = d.tl_c * zs - d.tl_s * xs;
                        xs = x1;
                    }
                    if (d.tilt_side) {
                        const double y1 = d.ts_c * ys - d.ts_s * zs;
                        zs = d.ts_s * ys + d.ts_c * zs;
                        ys = y1;
                    }
                    // Eq. (4): tool-centre offset; Eq. (7): half-open sampling boundaries
                    const double fx = ((xc[s] + xs) - x_lo) * inv;
                    const double fy = ((yq + ys) - y_lo) * inv;
                    if (fx >= 0.0 && fx < nxd && fy >= 0.0 && fy < nyd) {
                        const int64_t idx = (int64_t)(int32_t)fy * nx + (int32_t)fx;
                        const int64_t key = enc64(__double_as_longlong(zs));
                        if (key < __hip_atomic_load(zk + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                            __hip_atomic_fetch_min(zk + idx, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ++cnt;
                    }
                    m += spi;
                    while (m >= S) m -= S;
                }
            } else {
                const FSM_GLOBAL float *__restrict__ cs = gptr(d.csf + (size_t)K * S * 2);
                const FSM_GLOBAL float *ptf = gptr(d.pTf + ((size_t)K * d.N + p) * 4);
                const float px = ptf[0], py = ptf[1], pz = ptf[2];
                FSM_GLOBAL int32_t *__restrict__ zk = gptr(static_cast<int32_t *>(d.zmap));
                const float tlc = (float)d.tl_c, tls = (float)d.tl_s;
                const float tsc = (float)d.ts_c, tss = (float)d.ts_s;
                for (; s < s1; s += spi) {
                    const float ca = cs[2 * m], sa = cs[2 * m + 1];
                    float xs = fmaf(ca, px, sa * py);
                    float ys = fmaf(ca, py, -(sa * px));
                    float zs = pz;
                    if (d.tilt_lead) {
                        const float x1 = fmaf(tlc, xs, tls * zs);
                        zs = fmaf(tlc, zs, -(tls * xs));
                        xs = x1;
                    }
                    if (d.tilt_side) {
                        const float y1 = fmaf(tsc, ys, -(tss * zs));
                        zs = fmaf(tss, ys, tsc * zs);
                        ys = y1;
                    }
                    const double fx = ((xc[s] + (double)xs) - x_lo) * inv;
                    const double fy = ((yq + (double)ys) - y_lo) * inv;
                    if (fx >= 0.0 && fx < nxd && fy >= 0.0 && fy < nyd) {
                        const int64_t idx = (int64_t)(int32_t)fy * nx + (int32_t)fx;
                        const int32_t key = enc32(__float_as_int(zs));
                        if (key < __hip_atomic_load(zk + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                            __hip_atomic_fetch_min(zk + idx, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ++cnt;
                    }
                    m += spi;
                    while (m >= S) m -= S;
                }
            }
        }
    }
    const uint32_t tot = block_reduce(wave_sum(cnt), red, [](uint32_t a, uint32_t b) { return a + b; });
    if (tid == 0 && tot) atomicAdd((unsigned long long *)binned, (unsigned long long)tot);
}

// ---- binned Z-map ----------------------------------------------------------------------------
//
// The scatter form above touches one random cache line of the Z-map per binned point.  The
// binned form sorts the points by kTile x kTile cell tile first and reduces every tile in LDS:
//   count : per point, the tile it falls in; lanes are consecutive time steps, so equal tiles
//           come in runs and one atomic add per run counts them;
//   scan  : exclusive prefix sum of the counts -> bucket offsets (and write cursors);
//   write : the same points again, each run claiming its slots with one atomic add and every
//           lane storing (height key, cell index inside the tile);
//   reduce: one block per tile: keys in LDS, integer ds_min of every bucket entry, then one
//           coalesced store of the decoded tile (the Z-map is touched once per slice).

template <int PREC> struct KeyOf;
template <> struct KeyOf<FSM_F64> { using T = int64_t; static constexpr int64_t inf = kInf64; };
template <> struct KeyOf<FSM_F32> { using T = int32_t; static constexpr int32_t inf = kInf32; };

constexpr int kUnroll = 4;   // edge points in flight per lane

// Position of one edge point of the current (pass, step, tooth) in the workpiece frame and its
// bin.  Returns the global tile (or -1 outside the grid), the cell inside the tile and the key.
template <int PREC>
struct PointBin {
    int32_t tile;
    uint16_t cell;
    typename KeyOf<PREC>::T key;
};

template <int PREC>
__device__ __forceinline__ PointBin<PREC> bin_point(const DevSim &d, double ca, double sa,
                                                    float caf, float saf, double xcs, double yq,
                                                    int K, int p)
{
    PointBin<PREC> r;
    r.tile = -1;
    r.cell = 0;
    r.key = 0;
    double xs, ys;
    typename KeyOf<PREC>::T key;
    if (PREC == FSM_F64) {
        const FSM_GLOBAL double *pt = gptr(d.pT + ((size_t)K * d.N + p) * 3);
        const double xT = pt[0], yT = pt[1], zT = pt[2];
        // Eq. (3): [[c, s], [-s, c]] applied to the tool-frame point, then the tilt
        xs = ca * xT + sa * yT;
        ys = ca * yT - sa * xT;
        double zs = zT;
        if (d.tilt_lead) {
            const double x1 = d.tl_c * xs + d.tl_s * zs;
            zs = d.tl_c * zs - d.tl_s * xs;
            xs = x1;
        }
        if (d.tilt_side) {
            const double y1 = d.ts_c * ys - d.ts_s * zs;
            zs = d.ts_s * ys + d.ts_c * zs;
            ys = y1;
        }
        key = (typename KeyOf<PREC>::T)enc64(__double_as_longlong(zs));
    } else {
        const FSM_GLOBAL float *pt = gptr(d.pTf + ((size_t)K * d.N + p) * 4);
        const float px = pt[0], py = pt[1], pz = pt[2];
        float xf = fmaf(caf, px, saf * py);
        float yf = fmaf(caf, py, -(saf * px));
        float zf = pz;
        if (d.tilt_lead) {
            const float c = (float)d.tl_c, s = (float)d.tl_s;
            const float x1 = fmaf(c, xf, s * zf);
            zf = fmaf(c, zf, -(s * xf));
            xf = x1;
        }
        if (d.tilt_side) {
            const float c = (float)d.ts_c, s = (float)d.ts_s;
            const float y1 = fmaf(c, yf, -(s * zf));
            zf = fmaf(s, yf, c * zf);
            yf = y1;
        }
        xs = (double)xf;
        ys = (double)yf;
        key = (typename KeyOf<PREC>::T)enc32(__float_as_int(zf));
    }
    // Eq. (4): tool-centre offset; Eq. (7): half-open sampling boundaries
    const double fx = ((xcs + xs) - d.x_lo) * d.inv_dd;
    const double fy = ((yq + ys) - d.y_lo) * d.inv_dd;
    if (fx >= 0.0 && fx < d.nx_d && fy >= 0.0 && fy < d.ny_d) {
        const int32_t i = (int32_t)fx, j = (int32_t)fy;
        r.tile = (int32_t)d.tile_base + (j >> kTileShift) * d.tiles_x + (i >> kTileShift);
        r.cell = (uint16_t)(((j & (kTile - 1)) << kTileShift) | (i & (kTile - 1)));
        r.key = key;
    }
    return r;
}

// Runs of equal tiles over the 64 lanes of a wave.  head: first lane of a run; len: run
// length (valid in head lanes); first: head lane of this lane's run.
__device__ __forceinline__ void tile_runs(int32_t t, int lane, bool &head, int &len, int &first)
{
    int32_t prev = __shfl_up(t, 1, 64);
    if (lane == 0) prev = -2;
    head = t >= 0 && t != prev;
    const uint64_t heads = __ballot(head);
    const uint64_t ends = heads | __ballot(t < 0);
    const uint64_t le = (2ull << lane) - 1ull;
    const uint64_t above = ends & ~le;
    const int nxt = above ? __ffsll((unsigned long long)above) - 1 : 64;
    len = nxt - lane;
    const uint64_t mine = heads & le;
    first = mine ? 63 - __clzll((long long)mine) : lane;
}

template <int PREC, bool WRITE>
__global__ __launch_bounds__(kBlock) void bin_points(const DevSim *__restrict__ sims, int n_sims,
                                                     const int64_t *__restrict__ bitem_base,
                                                     int64_t item_begin, int64_t n_items,
                                                     uint32_t *__restrict__ counter,
                                                     void *__restrict__ bkey_v,
                                                     uint16_t *__restrict__ bidx, int64_t cap)
{
    using Key = typename KeyOf<PREC>::T;
    const int tid = threadIdx.x, lane = tid & 63;
    FSM_GLOBAL uint32_t *cnt = gptr(counter);
    FSM_GLOBAL Key *bkey = gptr(static_cast<Key *>(bkey_v));
    FSM_GLOBAL uint16_t *bix = gptr(bidx);
    for (int64_t b = blockIdx.x; b < n_items; b += gridDim.x) {
        const int64_t round0 = b - blockIdx.x;
        const int64_t rn = n_items - round0 < (int64_t)gridDim.x ? n_items - round0 : (int64_t)gridDim.x;
        const int64_t item = item_begin + round0 + xcd_item(b - round0, rn);
        const int si = n_sims == 1 ? 0 : find_sim(bitem_base, n_sims, item);
        const DevSim d = sims[si];
        int64_t local = item - d.bitem_base;
        const int K = (int)(local % d.z_n);
        local /= d.z_n;
        const int sb = (int)(local % d.n_sblocks);
        const int q = (int)(local / d.n_sblocks);
        const int s = sb * kBlock + tid;
        const bool vs = s < d.n_steps;
        double ca = 0.0, sa = 0.0, xcs = 0.0;
        float caf = 0.0f, saf = 0.0f;
        if (vs) {
            const int m = s % d.S;
            if (PREC == FSM_F64) {
                const FSM_GLOBAL double *cs = gptr(d.cs + ((size_t)K * d.S + m) * 2);
                ca = cs[0];
                sa = cs[1];
            } else {
                const FSM_GLOBAL float *cs = gptr(d.csf + ((size_t)K * d.S + m) * 2);
                caf = cs[0];
                saf = cs[1];
            }
            xcs = gptr(d.xc)[s];
        }
        const double yq = d.y_first + (double)q * d.a_e;
        for (int p0 = 0; p0 < d.N; p0 += kUnroll) {
            PointBin<PREC> pb[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                pb[u].tile = -1;
                if (vs && p0 + u < d.N) pb[u] = bin_point<PREC>(d, ca, sa, caf, saf, xcs, yq, K, p0 + u);
            }
            bool head[kUnroll];
            int len[kUnroll], first[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) tile_runs(pb[u].tile, lane, head[u], len[u], first[u]);
            if (!WRITE) {
#pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    if (head[u]) __hip_atomic_fetch_add(cnt + pb[u].tile, (uint32_t)len[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                uint32_t base[kUnroll];
#pragma unroll
                for (int u = 0; u < kUnroll; ++u)
                    base[u] = head[u] ? __hip_atomic_fetch_add(cnt + pb[u].tile, (uint32_t)len[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    const uint32_t b0 = __shfl(base[u], first[u], 64);
                    if (pb[u].tile >= 0) {
                        const int64_t pos = (int64_t)b0 + (lane - first[u]);
                        if (pos < cap) {
                            bkey[pos] = pb[u].key;
                            bix[pos] = pb[u].cell;
                        }
                    }
                }
            }
        }
    }
}

// Exclusive scan of the tile counts in three launches: per-block sums of kScanSeg counts, a
// one-block scan of those sums (also adds the slice total to the in-grid counter), and the
// per-block scan that writes offsets and cursors.
constexpr int kScanSeg = 4096;
constexpr int kScanPer = kScanSeg / kBlock;   // counts per thread

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

__global__ __launch_bounds__(kBlock) void scan_top(uint32_t *bsum, int nb, uint32_t *offsets, int64_t n,
                                                  uint64_t *binned)
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
    if (threadIdx.x == 0) {
        offsets[n] = carry;
        if (binned) *binned += carry;
    }
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

template <int PREC>
__global__ __launch_bounds__(kBlock) void tile_reduce(const DevSim *__restrict__ sims, int n_sims,
                                                      const int64_t *__restrict__ tile_base,
                                                      int64_t n_tiles, const uint32_t *__restrict__ offsets,
                                                      const void *__restrict__ bkey_v,
                                                      const uint16_t *__restrict__ bidx, int first_slice)
{
    using Key = typename KeyOf<PREC>::T;
    __shared__ Key lds[kTile * kTile];
    const FSM_GLOBAL Key *bkey = gptr(static_cast<const Key *>(bkey_v));
    const FSM_GLOBAL uint16_t *bix = gptr(bidx);
    const int tid = threadIdx.x;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int si = n_sims == 1 ? 0 : find_sim(tile_base, n_sims, t);
        const DevSim d = sims[si];
        const int64_t lt = t - d.tile_base;
        const int tx = (int)(lt % d.tiles_x), ty = (int)(lt / d.tiles_x);
        const int64_t i0 = (int64_t)tx << kTileShift, j0 = (int64_t)ty << kTileShift;
        const int w = d.nx - i0 < kTile ? (int)(d.nx - i0) : kTile;
        const int h = d.ny - j0 < kTile ? (int)(d.ny - j0) : kTile;
        FSM_GLOBAL Key *Z = gptr(static_cast<Key *>(d.zmap)) + j0 * d.nx + i0;
        for (int l = tid; l < kTile * kTile; l += kBlock) {
            const int li = l & (kTile - 1), lj = l >> kTileShift;
            Key v = KeyOf<PREC>::inf;
            if (!first_slice && li < w && lj < h) {
                const Key zb = Z[(int64_t)lj * d.nx + li];
                v = PREC == FSM_F64 ? (Key)enc64((int64_t)zb) : (Key)enc32((int32_t)zb);
            }
            lds[l] = v;
        }
        __syncthreads();
        const uint32_t e1 = offsets[t + 1];
        for (uint32_t e = offsets[t] + tid; e < e1; e += kBlock)
            __hip_atomic_fetch_min(&lds[bix[e]], bkey[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
        for (int l = tid; l < kTile * kTile; l += kBlock) {
            const int li = l & (kTile - 1), lj = l >> kTileShift;
            if (li < w && lj < h) {
                const Key k = lds[l];
                Z[(int64_t)lj * d.nx + li] = PREC == FSM_F64 ? (Key)enc64((int64_t)k) : (Key)enc32((int32_t)k);
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void zero_u32(uint32_t *p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) p[k] = 0u;
}

// ---- roughness -------------------------------------------------------------------------------

// Height of one Z-map element; decodes the scatter's integer keys when `decode` is set.
__device__ __forceinline__ double height64(int64_t k, bool decode)
{
    return __longlong_as_double(decode ? enc64(k) : k);
}
__device__ __forceinline__ double height32(int32_t k, bool decode)
{
    return (double)__int_as_float(decode ? enc32(k) : k);
}

struct Acc1 {
    double sum = 0.0, mn = INFINITY, mx = -INFINITY;
    int64_t n = 0;
    __device__ void add(double v)
    {
        if (v < INFINITY) {
            sum += v;
            mn = fmin(mn, v);
            mx = fmax(mx, v);
            ++n;
        }
    }
};

__device__ void store_part1(Acc1 a, RoughPart1 *part)
{
    __shared__ double bd[4];
    __shared__ int64_t bn[4];
    const double s = block_reduce(wave_sum(a.sum), bd, [](double x, double y) { return x + y; });
    const double mn = block_reduce(wave_min(a.mn), bd, [](double x, double y) { return fmin(x, y); });
    const double mx = block_reduce(wave_max(a.mx), bd, [](double x, double y) { return fmax(x, y); });
    const int64_t n = block_reduce(wave_sum(a.n), bn, [](int64_t x, int64_t y) { return x + y; });
    if (threadIdx.x == 0) part[blockIdx.x] = RoughPart1{s, mn, mx, n};
}

// Pass 1: count, sum, min, max of the reached cells.  With `decode`, integer keys left by the
// scatter become heights; only negative heights change bits, so only those are written back.
template <int PREC>
__global__ __launch_bounds__(kBlock) void rough1(void *zmap, int64_t n, bool decode, RoughPart1 *part)
{
    Acc1 a;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (PREC == FSM_F64) {
        int64_t *z = static_cast<int64_t *>(zmap);
        const int64_t n2 = n >> 1;
        for (int64_t k = gid; k < n2; k += stride) {
            longlong2 v = reinterpret_cast<longlong2 *>(z)[k];
            if (decode && (v.x < 0 || v.y < 0)) {
                reinterpret_cast<longlong2 *>(z)[k] = longlong2{enc64(v.x), enc64(v.y)};
            }
            a.add(height64(v.x, decode));
            a.add(height64(v.y, decode));
        }
        if ((n & 1) && gid == 0) {
            const int64_t v = z[n - 1];
            if (decode && v < 0) z[n - 1] = enc64(v);
            a.add(height64(v, decode));
        }
    } else {
        int32_t *z = static_cast<int32_t *>(zmap);
        const int64_t n4 = n >> 2;
        for (int64_t k = gid; k < n4; k += stride) {
            int4 v = reinterpret_cast<int4 *>(z)[k];
            if (decode && (v.x < 0 || v.y < 0 || v.z < 0 || v.w < 0)) {
                reinterpret_cast<int4 *>(z)[k] = int4{enc32(v.x), enc32(v.y), enc32(v.z), enc32(v.w)};
            }
            a.add(height32(v.x, decode));
            a.add(height32(v.y, decode));
            a.add(height32(v.z, decode));
            a.add(height32(v.w, decode));
        }
        if (gid < (n & 3)) {
            const int64_t k = (n4 << 2) + gid;
            const int32_t v = z[k];
            if (decode && v < 0) z[k] = enc32(v);
            a.add(height32(v, decode));
        }
    }
    store_part1(a, part);
}

__device__ __forceinline__ double load_height(const void *zmap, int64_t k, int prec)
{
    return prec == FSM_F64 ? static_cast<const double *>(zmap)[k]
                           : (double)static_cast<const float *>(zmap)[k];
}

// Sum and count of the reached cells along a line (start, stride, count), block-wide.
__device__ void line_sum(const void *zmap, int prec, int64_t start, int64_t stride, int64_t cnt,
                         double &sum, int64_t &n)
{
    __shared__ double bd[4];
    __shared__ int64_t bn[4];
    double s = 0.0;
    int64_t m = 0;
    for (int64_t k = threadIdx.x; k < cnt; k += kBlock) {
        const double v = load_height(zmap, start + k * stride, prec);
        if (v < INFINITY) { s += v; ++m; }
    }
    sum = block_reduce(wave_sum(s), bd, [](double x, double y) { return x + y; });
    n = block_reduce(wave_sum(m), bn, [](int64_t x, int64_t y) { return x + y; });
}

__device__ double line_absdev(const void *zmap, int prec, int64_t start, int64_t stride,
                              int64_t cnt, double mu)
{
    __shared__ double bd[4];
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < cnt; k += kBlock) {
        const double v = load_height(zmap, start + k * stride, prec);
        if (v < INFINITY) s += fabs(v - mu);
    }
    return block_reduce(wave_sum(s), bd, [](double x, double y) { return x + y; });
}

// One block: combine the pass-1 partials in a fixed order and the two profile means.
__global__ __launch_bounds__(kBlock) void rough1_final(const void *zmap, int prec, int64_t nx, int64_t ny,
                                                      const RoughPart1 *part, int nparts, RoughState *st)
{
    Acc1 a;
    for (int k = threadIdx.x; k < nparts; k += kBlock) {
        const RoughPart1 p = part[k];
        a.sum += p.sum;
        a.mn = fmin(a.mn, p.mn);
        a.mx = fmax(a.mx, p.mx);
        a.n += p.n;
    }
    __shared__ double bd[4];
    __shared__ int64_t bn[4];
    const double sum = block_reduce(wave_sum(a.sum), bd, [](double x, double y) { return x + y; });
    const double mn = block_reduce(wave_min(a.mn), bd, [](double x, double y) { return fmin(x, y); });
    const double mx = block_reduce(wave_max(a.mx), bd, [](double x, double y) { return fmax(x, y); });
    const int64_t n = block_reduce(wave_sum(a.n), bn, [](int64_t x, int64_t y) { return x + y; });
    double rs, cs;
    int64_t rn, cn;
    line_sum(zmap, prec, (ny / 2) * nx, 1, nx, rs, rn);
    line_sum(zmap, prec, nx / 2, nx, ny, cs, cn);
    if (threadIdx.x == 0) {
        st->n = n;
        st->mean = n ? sum / (double)n : NAN;
        st->mn = mn;
        st->mx = mx;
        st->n_row = rn;
        st->row_mean = rn ? rs / (double)rn : NAN;
        st->n_col = cn;
        st->col_mean = cn ? cs / (double)cn : NAN;
    }
}

struct Acc2 {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    __device__ void add(double v, double mu)
    {
        if (v < INFINITY) {
            const double d = v - mu;
            const double d2 = d * d;
            s1 += fabs(d);
            s2 += d2;
            s3 += d2 * d;
            s4 += d2 * d2;
        }
    }
};

// Pass 2: central moments about the mean of pass 1.
template <int PREC>
__global__ __launch_bounds__(kBlock) void rough2(const void *zmap, int64_t n, const RoughState *st, RoughPart2 *part)
{
    const double mu = st->mean;
    Acc2 a;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (PREC == FSM_F64) {
        const double *z = static_cast<const double *>(zmap);
        const int64_t n2 = n >> 1;
        for (int64_t k = gid; k < n2; k += stride) {
            const double2 v = reinterpret_cast<const double2 *>(z)[k];
            a.add(v.x, mu);
            a.add(v.y, mu);
        }
        if ((n & 1) && gid == 0) a.add(z[n - 1], mu);
    } else {
        const float *z = static_cast<const float *>(zmap);
        const int64_t n4 = n >> 2;
        for (int64_t k = gid; k < n4; k += stride) {
            const float4 v = reinterpret_cast<const float4 *>(z)[k];
            a.add(v.x, mu);
            a.add(v.y, mu);
            a.add(v.z, mu);
            a.add(v.w, mu);
        }
        if (gid < (n & 3)) a.add(z[(n4 << 2) + gid], mu);
    }
    __shared__ double bd[4];
    const double s1 = block_reduce(wave_sum(a.s1), bd, [](double x, double y) { return x + y; });
    const double s2 = block_reduce(wave_sum(a.s2), bd, [](double x, double y) { return x + y; });
    const double s3 = block_reduce(wave_sum(a.s3), bd, [](double x, double y) { return x + y; });
    const double s4 = block_reduce(wave_sum(a.s4), bd, [](double x, double y) { return x + y; });
    if (threadIdx.x == 0) part[blockIdx.x] = RoughPart2{s1, s2, s3, s4};
}

// One block: combine the pass-2 partials and write the result record.
__global__ __launch_bounds__(kBlock) void rough2_final(const void *zmap, int prec, int64_t nx, int64_t ny,
                                                      const RoughPart2 *part, int nparts,
                                                      const RoughState *st, const uint64_t *binned,
                                                      int64_t n_evals, fsm_rough *out)
{
    Acc2 a;
    for (int k = threadIdx.x; k < nparts; k += kBlock) {
        const RoughPart2 p = part[k];
        a.s1 += p.s1;
        a.s2 += p.s2;
        a.s3 += p.s3;
        a.s4 += p.s4;
    }
    __shared__ double bd[4];
    const double s1 = block_reduce(wave_sum(a.s1), bd, [](double x, double y) { return x + y; });
    const double s2 = block_reduce(wave_sum(a.s2), bd, [](double x, double y) { return x + y; });
    const double s3 = block_reduce(wave_sum(a.s3), bd, [](double x, double y) { return x + y; });
    const double s4 = block_reduce(wave_sum(a.s4), bd, [](double x, double y) { return x + y; });
    const double ra_row = line_absdev(zmap, prec, (ny / 2) * nx, 1, nx, st->row_mean);
    const double ra_col = line_absdev(zmap, prec, nx / 2, nx, ny, st->col_mean);
    if (threadIdx.x == 0) {
        fsm_rough r;
        const int64_t n = st->n;
        const double dn = (double)n;
        const double mu = st->mean;
        r.n_hit = n;
        r.n_evals = n_evals;
        r.n_binned = binned ? (int64_t)*binned : 0;
        r.n_feed = st->n_row;
        r.n_pick = st->n_col;
        r.flags = 0;
        r.reserved = 0;
        r.mean = mu;
        if (n == 0) {
            r.Sa = r.Sq = r.Sp = r.Sv = r.Sz = r.Ssk = r.Sku = NAN;
            r.flags |= FSM_FLAG_NO_HIT;
        } else {
            r.Sa = s1 / dn;
            r.Sq = sqrt(s2 / dn);
            r.Sp = st->mx - mu;
            r.Sv = mu - st->mn;
            r.Sz = r.Sp + r.Sv;
            if (r.Sq > 0.0) {
                r.Ssk = (s3 / dn) / (r.Sq * r.Sq * r.Sq);
                r.Sku = (s4 / dn) / (r.Sq * r.Sq * r.Sq * r.Sq);
            } else {
                r.Ssk = r.Sku = NAN;
                r.flags |= FSM_FLAG_SQ_ZERO;
            }
        }
        if ((double)n < 0.99 * (double)nx * (double)ny) r.flags |= FSM_FLAG_LOW_COVERAGE;
        r.Ra_feed = st->n_row ? ra_row / (double)st->n_row : NAN;
        r.Ra_pick = st->n_col ? ra_col / (double)st->n_col : NAN;
        *out = r;
    }
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void decode_only(void *zmap, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += stride) {
        if (PREC == FSM_F64) {
            int64_t *z = static_cast<int64_t *>(zmap);
            const int64_t v = z[k];
            if (v < 0) z[k] = enc64(v);
        } else {
            int32_t *z = static_cast<int32_t *>(zmap);
            const int32_t v = z[k];
            if (v < 0) z[k] = enc32(v);
        }
    }
}

int stream_blocks(int64_t work, int64_t per_block, int cap)
{
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

}  // namespace

int launch_fill(void *zmap, int64_t n, int precision, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int blocks = stream_blocks(n, (int64_t)kBlock * 8, 8192);
    if (precision == FSM_F64)
        hipLaunchKernelGGL(fill64, dim3(blocks), dim3(kBlock), 0, s, static_cast<int64_t *>(zmap), n);
    else
        hipLaunchKernelGGL(fill32, dim3(blocks), dim3(kBlock), 0, s, static_cast<int32_t *>(zmap), n);
    return (int)hipGetLastError();
}

int launch_scatter(const DevSim *d_sims, const DevSim &, int64_t n_items, int n_sims,
                   const int64_t *d_item_base, int precision, uint64_t *d_binned, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t cap = (int64_t)1 << 20;
    const int blocks = (int)(n_items < cap ? n_items : cap);
    if (blocks <= 0) return 0;
    if (precision == FSM_F64)
        hipLaunchKernelGGL(scatter<FSM_F64>, dim3(blocks), dim3(kBlock), 0, s, d_sims, n_sims, d_item_base, n_items, d_binned);
    else
        hipLaunchKernelGGL(scatter<FSM_F32>, dim3(blocks), dim3(kBlock), 0, s, d_sims, n_sims, d_item_base, n_items, d_binned);
    return (int)hipGetLastError();
}

int launch_rough(void *zmap, int64_t nx, int64_t ny, int precision, bool decode,
                 RoughPart1 *p1, RoughPart2 *p2, RoughState *st, fsm_rough *d_out,
                 const uint64_t *d_binned, int64_t n_evals, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = nx * ny;
    const int blocks = stream_blocks(n, (int64_t)kBlock * 4, kRoughBlocks);
    if (precision == FSM_F64) {
        hipLaunchKernelGGL(rough1<FSM_F64>, dim3(blocks), dim3(kBlock), 0, s, zmap, n, decode, p1);
        hipLaunchKernelGGL(rough1_final, dim3(1), dim3(kBlock), 0, s, (const void *)zmap, precision, nx, ny, (const RoughPart1 *)p1, blocks, st);
        hipLaunchKernelGGL(rough2<FSM_F64>, dim3(blocks), dim3(kBlock), 0, s, (const void *)zmap, n, (const RoughState *)st, p2);
    } else {
        hipLaunchKernelGGL(rough1<FSM_F32>, dim3(blocks), dim3(kBlock), 0, s, zmap, n, decode, p1);
        hipLaunchKernelGGL(rough1_final, dim3(1), dim3(kBlock), 0, s, (const void *)zmap, precision, nx, ny, (const RoughPart1 *)p1, blocks, st);
        hipLaunchKernelGGL(rough2<FSM_F32>, dim3(blocks), dim3(kBlock), 0, s, (const void *)zmap, n, (const RoughState *)st, p2);
    }
    hipLaunchKernelGGL(rough2_final, dim3(1), dim3(kBlock), 0, s, (const void *)zmap, precision, nx, ny,
                       (const RoughPart2 *)p2, blocks, (const RoughState *)st, d_binned, n_evals, d_out);
    return (int)hipGetLastError();
}

int launch_decode(void *zmap, int64_t n, int precision, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int blocks = stream_blocks(n, (int64_t)kBlock * 8, 8192);
    if (precision == FSM_F64)
        hipLaunchKernelGGL(decode_only<FSM_F64>, dim3(blocks), dim3(kBlock), 0, s, zmap, n);
    else
        hipLaunchKernelGGL(decode_only<FSM_F32>, dim3(blocks), dim3(kBlock), 0, s, zmap, n);
    return (int)hipGetLastError();
}

int launch_binned_slice(const DevSim *d_sims, int n_sims, const int64_t *d_bitem_base,
                        const int64_t *d_tile_base, int64_t n_tiles, int64_t item_begin,
                        int64_t n_items, const BinBuffers &bb, bool first_slice,
                        int precision, uint64_t *d_binned, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int zb = stream_blocks(n_tiles, kBlock, 4096);
    hipLaunchKernelGGL(zero_u32, dim3(zb), dim3(kBlock), 0, s, bb.counts, n_tiles);
    const int64_t cap_blocks = (int64_t)1 << 20;
    const int ib = (int)(n_items < cap_blocks ? n_items : cap_blocks);
    const int nb = (int)((n_tiles + kScanSeg - 1) / kScanSeg);
    // block sums of the scan live after the cursor array
    uint32_t *bsum = bb.cursor + n_tiles;
    const int tb = (int)(n_tiles < cap_blocks ? n_tiles : cap_blocks);
    if (precision == FSM_F64) {
        if (ib > 0)
            hipLaunchKernelGGL((bin_points<FSM_F64, false>), dim3(ib), dim3(kBlock), 0, s, d_sims, n_sims, d_bitem_base, item_begin, n_items, bb.counts, bb.bkey, bb.bidx, bb.cap);
        hipLaunchKernelGGL(scan_reduce, dim3(nb), dim3(kBlock), 0, s, (const uint32_t *)bb.counts, n_tiles, bsum);
        hipLaunchKernelGGL(scan_top, dim3(1), dim3(kBlock), 0, s, bsum, nb, bb.offsets, n_tiles, d_binned);
        hipLaunchKernelGGL(scan_apply, dim3(nb), dim3(kBlock), 0, s, (const uint32_t *)bb.counts, n_tiles, (const uint32_t *)bsum, bb.offsets, bb.cursor);
        if (ib > 0)
            hipLaunchKernelGGL((bin_points<FSM_F64, true>), dim3(ib), dim3(kBlock), 0, s, d_sims, n_sims, d_bitem_base, item_begin, n_items, bb.cursor, bb.bkey, bb.bidx, bb.cap);
        hipLaunchKernelGGL(tile_reduce<FSM_F64>, dim3(tb), dim3(kBlock), 0, s, d_sims, n_sims, d_tile_base, n_tiles, (const uint32_t *)bb.offsets, (const void *)bb.bkey, (const uint16_t *)bb.bidx, first_slice ? 1 : 0);
    } else {
        if (ib > 0)
            hipLaunchKernelGGL((bin_points<FSM_F32, false>), dim3(ib), dim3(kBlock), 0, s, d_sims, n_sims, d_bitem_base, item_begin, n_items, bb.counts, bb.bkey, bb.bidx, bb.cap);
        hipLaunchKernelGGL(scan_reduce, dim3(nb), dim3(kBlock), 0, s, (const uint32_t *)bb.counts, n_tiles, bsum);
        hipLaunchKernelGGL(scan_top, dim3(1), dim3(kBlock), 0, s, bsum, nb, bb.offsets, n_tiles, d_binned);
        hipLaunchKernelGGL(scan_apply, dim3(nb), dim3(kBlock), 0, s, (const uint32_t *)bb.counts, n_tiles, (const uint32_t *)bsum, bb.offsets, bb.cursor);
        if (ib > 0)
            hipLaunchKernelGGL((bin_points<FSM_F32, true>), dim3(ib), dim3(kBlock), 0, s, d_sims, n_sims, d_bitem_base, item_begin, n_items, bb.cursor, bb.bkey, bb.bidx, bb.cap);
        hipLaunchKernelGGL(tile_reduce<FSM_F32>, dim3(tb), dim3(kBlock), 0, s, d_sims, n_sims, d_tile_base, n_tiles, (const uint32_t *)bb.offsets, (const void *)bb.bkey, (const uint16_t *)bb.bidx, first_slice ? 1 : 0);
    }
    return (int)hipGetLastError();
}

}  // namespace fsm
