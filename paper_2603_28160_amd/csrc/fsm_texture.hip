// fsm_texture.hip -- gfx950 kernels of the surface-texture operators applied to a Z-map: the
// S-filter, F-operator and L-filter under which the paper's measured topographies were taken
// (Sec. 4.1.1), so that a predicted map can be evaluated the same way.
//
//   plane  : least-squares plane over the hit cells.  Per block, FP64 moments of the design
//            rows (1, u, v) and of z, with (u, v) the cell's column and row measured from the
//            grid's centre (exact integers, so the normal matrix is exact for maps up to ~1e8
//            cells); one block combines the block partials in a fixed order and solves the
//            3 x 3 normal equations; a third kernel subtracts the plane.
//   gauss  : separable normalised Gaussian, out = sum(w z h) / sum(w h) over the square window
//            (h = 1 on hit cells), every product of the 2-D weight being w(dx) w(dy):
//            rows - one block per (row, 1024-column tile); the tile and its halo in LDS
//                   (skewed by one slot per eight against bank conflicts); each lane owns
//                   eight consecutive outputs and slides a register window over the taps,
//                   so each LDS value feeds sixteen fused multiply-adds; weights are wave-
//                   uniform scalar loads.  Writes (numerator, denominator) pairs.
//            cols - lanes along the row (coalesced 16-byte pair loads from L2), each lane owns
//                   sixteen consecutive rows of one column and accumulates every input row
//                   into all sixteen outputs with a scalar weight each; then the quotient,
//                   or the input minus it, is stored, empty cells stay +inf.
//
// All arithmetic is FP64 (both map precisions: single-precision maps are widened on load and
// rounded once on store).  Without packed FP32 the FP64 and FP32 FMA rates are equal here, so
// the wider type costs only LDS and L2 bytes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "fsm_internal.h"

namespace fsm {

namespace {

constexpr int kRowThreads = 128;
constexpr int kRowOut = 8;
constexpr int kRowTile = kRowThreads * kRowOut;   // outputs per row block
constexpr int kColOut = 16;                       // rows per lane in the column pass
constexpr int kColWaves = 4;
constexpr int kColRows = kColWaves * kColOut;     // rows per column block
constexpr int kPlaneBlocks = kPlanePartials / 9;
constexpr int64_t kMaxItems = 1 << 20;

__device__ __forceinline__ bool is_hit(double v) { return v < INFINITY; }

__device__ __forceinline__ int skew(int p) { return p + (p >> 3); }

template <typename T> __device__ __forceinline__ T inf_of();
template <> __device__ __forceinline__ double inf_of<double>() { return INFINITY; }
template <> __device__ __forceinline__ float inf_of<float>() { return INFINITY; }

// Sum of v over the 256 threads of a block; every thread gets the result.  Fixed order.
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// ---- F-operator ------------------------------------------------------------------------------

// Block partials of (n, su, sv, suu, suv, svv, sz, suz, svz) of map blockIdx.y over rows
// blockIdx.x, +gridDim.x, ...
template <typename T>
__global__ void __launch_bounds__(256) plane_moments(const T *const *__restrict__ zs, int64_t nx, int64_t ny,
                                                     double ci, double cj, double *__restrict__ part)
{
    __shared__ double sh[4];
    const T *__restrict__ z = zs[blockIdx.y];
    part += (int64_t)blockIdx.y * gridDim.x * 9;
    double a[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t j = blockIdx.x; j < ny; j += gridDim.x) {
        const double v = (double)j - cj;
        for (int64_t i = threadIdx.x; i < nx; i += blockDim.x) {
            const double h = (double)z[j * nx + i];
            if (!is_hit(h)) continue;
            const double u = (double)i - ci;
            a[0] += 1.0;
            a[1] += u;
            a[2] += v;
            a[3] += u * u;
            a[4] += u * v;
            a[5] += v * v;
            a[6] += h;
            a[7] += u * h;
            a[8] += v * h;
        }
    }
    for (int q = 0; q < 9; ++q) {
        const double s = block_sum(a[q], sh);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 9 + q] = s;
    }
}

// One block per map: combine its nb partials in block order and solve the normal equations by
// Gaussian elimination with partial pivoting.  coef[4 map ..] = (c0, cu, cv, status): z ~ c0 +
// cu u + cv v; status 1, or 0 for fewer than three hit cells or hit cells on one line (a pivot
// that vanishes relative to its column's diagonal).
__global__ void __launch_bounds__(256) plane_solve(const double *__restrict__ part, int nb,
                                                   double *__restrict__ coef)
{
    __shared__ double sh[4];
    __shared__ double m[9];
    part += (int64_t)blockIdx.x * nb * 9;
    coef += (int64_t)blockIdx.x * 4;
    for (int q = 0; q < 9; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[(int64_t)b * 9 + q];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) m[q] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double M[3][4] = {{m[0], m[1], m[2], m[6]}, {m[1], m[3], m[4], m[7]}, {m[2], m[4], m[5], m[8]}};
    const double diag[3] = {m[0], m[3], m[5]};
    bool ok = m[0] >= 3.0;
    for (int col = 0; col < 3 && ok; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (!(fabs(M[piv][col]) > 1e-10 * diag[col])) { ok = false; break; }
        if (piv != col)
            for (int k = 0; k < 4; ++k) {
                const double t = M[col][k];
                M[col][k] = M[piv][k];
                M[piv][k] = t;
            }
        for (int r = col + 1; r < 3; ++r) {
            const double f = M[r][col] / M[col][col];
            for (int k = col; k < 4; ++k) M[r][k] -= f * M[col][k];
        }
    }
    double c[3] = {0.0, 0.0, 0.0};
    if (ok)
        for (int r = 2; r >= 0; --r) {
            double v = M[r][3];
            for (int k = r + 1; k < 3; ++k) v -= M[r][k] * c[k];
            c[r] = v / M[r][r];
        }
    coef[0] = c[0];
    coef[1] = c[1];
    coef[2] = c[2];
    coef[3] = ok ? 1.0 : 0.0;
}

// out = z - plane on hit cells (+inf elsewhere) of map blockIdx.y; a degenerate fit leaves the
// values as they are.
template <typename T>
__global__ void __launch_bounds__(256) plane_apply(const T *const *zs, T *const *outs, int64_t nx, int64_t ny,
                                                   double ci, double cj, const double *__restrict__ coef)
{
    const T *z = zs[blockIdx.y];
    T *out = outs[blockIdx.y];
    coef += (int64_t)blockIdx.y * 4;
    const double c0 = coef[0], cu = coef[1], cv = coef[2];
    const bool ok = coef[3] != 0.0;
    for (int64_t j = blockIdx.x; j < ny; j += gridDim.x) {
        const double v = (double)j - cj;
        for (int64_t i = threadIdx.x; i < nx; i += blockDim.x) {
            const int64_t k = j * nx + i;
            const double h = (double)z[k];
            double r = h;
            if (ok && is_hit(h)) r = h - ((c0 + cu * ((double)i - ci)) + cv * v);
            out[k] = is_hit(h) ? (T)r : inf_of<T>();
        }
    }
}

// ---- Gaussian filter -------------------------------------------------------------------------

// flag = 1 if any cell of the map is empty (flag zeroed by the first kernel of the pair).
__global__ void clear_flag(int *flag) { *flag = 0; }

template <typename T>
__global__ void __launch_bounds__(256) scan_holes(const T *const *__restrict__ zs, int64_t n, int *flag)
{
    const T *__restrict__ z = zs[blockIdx.y];
    // the flag only ever goes from 0 to 1: once it is set, nothing is left to find (one
    // thread reads it and the whole block follows, so every thread reaches the barriers)
    if (__syncthreads_or(threadIdx.x == 0 && __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0))
        return;
    int any = 0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
        any |= is_hit((double)z[k]) ? 0 : 1;
    if (__syncthreads_or(any) && threadIdx.x == 0 &&
        __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        atomicOr(flag, 1);
}

// Row pass.  g[k] = w(|k - R|) for k <= 2R, zero up to K8 (a multiple of eight).
// HOLES: nd[j][i] = (sum_k g[k] zh(i - R + k), sum_k g[k] h(i - R + k)) as double2 pairs.
// Without holes (every cell hit) the denominator is separable and known (the caller's
// per-column and per-row weight sums), so only the numerator is summed and stored (double).
template <typename T, bool HOLES>
__global__ void __launch_bounds__(kRowThreads) gauss_rows(const T *const *__restrict__ zs, int64_t nx, int64_t ny,
                                                          int R, int K8, const double *__restrict__ g,
                                                          double *__restrict__ nd)
{
    extern __shared__ double lds[];
    const T *__restrict__ z = zs[blockIdx.y];
    nd += (int64_t)blockIdx.y * nx * ny * (HOLES ? 2 : 1);
    const int64_t tiles = (nx + kRowTile - 1) / kRowTile;
    const int L = kRowTile + K8 + 8;
    const int b = threadIdx.x * kRowOut;
    // outside the grid: empty with holes; a zero that adds nothing without
    const double outside = HOLES ? INFINITY : 0.0;
    for (int64_t item = blockIdx.x; item < tiles * ny; item += gridDim.x) {
        const int64_t j = item / tiles, tx = item - j * tiles;
        const int64_t x0 = tx * kRowTile - R;        // grid column of LDS position 0
        const T *row = z + j * nx;
        __syncthreads();
        for (int p = threadIdx.x; p < L; p += kRowThreads) {
            const int64_t c = x0 + p;
            lds[skew(p)] = (c >= 0 && c < nx) ? (double)row[c] : outside;
        }
        __syncthreads();
        double an[kRowOut], ad[kRowOut], cz[2 * kRowOut], ch[2 * kRowOut];
#pragma unroll
        for (int o = 0; o < kRowOut; ++o) {
            an[o] = 0.0;
            ad[o] = 0.0;
            const double v = lds[skew(b + o)];
            if (HOLES) {
                ch[o] = is_hit(v) ? 1.0 : 0.0;
                cz[o] = is_hit(v) ? v : 0.0;
            } else {
                cz[o] = v;
            }
        }
        for (int k0 = 0; k0 < K8; k0 += kRowOut) {
#pragma unroll
            for (int o = 0; o < kRowOut; ++o) {
                const double v = lds[skew(b + k0 + kRowOut + o)];
                if (HOLES) {
                    ch[kRowOut + o] = is_hit(v) ? 1.0 : 0.0;
                    cz[kRowOut + o] = is_hit(v) ? v : 0.0;
                } else {
                    cz[kRowOut + o] = v;
                }
            }
#pragma unroll
            for (int u = 0; u < kRowOut; ++u) {
                const double w = g[k0 + u];
#pragma unroll
                for (int o = 0; o < kRowOut; ++o) {
                    an[o] = fma(w, cz[u + o], an[o]);
                    if (HOLES) ad[o] = fma(w, ch[u + o], ad[o]);
                }
            }
#pragma unroll
            for (int o = 0; o < kRowOut; ++o) {
                cz[o] = cz[kRowOut + o];
                if (HOLES) ch[o] = ch[kRowOut + o];
            }
        }
        const int64_t c0 = tx * kRowTile + b;
#pragma unroll
        for (int o = 0; o < kRowOut; ++o) {
            if (c0 + o >= nx) continue;
            if (HOLES)
                reinterpret_cast<double2 *>(nd)[j * nx + c0 + o] = make_double2(an[o], ad[o]);
            else
                nd[j * nx + c0 + o] = an[o];
        }
    }
}

// Column pass.  gc[16 + k] = w(|k - R|) for k in [0, 2R], zero in the 16 slots on either
// side.  Lane i of wave w in block (tx, ty) owns rows j0 .. j0 + 15 of column tx*64 + lane,
// j0 = ty*64 + 16 w (kColRows = 64 rows per block).  Without holes the denominator of cell
// (i, j) is cx[i] cy[j], the sums of the weights whose cells lie inside the grid.
template <typename T, bool HOLES>
__global__ void __launch_bounds__(64 * kColWaves) gauss_cols(const T *const *zs, T *const *outs, int64_t nx, int64_t ny,
                                                             int R, const double *__restrict__ gc,
                                                             const double *__restrict__ cx,
                                                             const double *__restrict__ cy,
                                                             const double *__restrict__ nd, int mode)
{
    const T *z = zs[blockIdx.y];
    T *out = outs[blockIdx.y];
    nd += (int64_t)blockIdx.y * nx * ny * (HOLES ? 2 : 1);
    const int64_t tiles_x = (nx + 63) / 64, tiles_y = (ny + kColRows - 1) / kColRows;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t item = blockIdx.x; item < tiles_x * tiles_y; item += gridDim.x) {
        const int64_t ty = item / tiles_x, tx = item - ty * tiles_x;
        const int64_t i = tx * 64 + lane;
        const int64_t j0 = ty * kColRows + (int64_t)wave * kColOut;
        if (j0 >= ny) continue;
        double an[kColOut], ad[kColOut];
#pragma unroll
        for (int o = 0; o < kColOut; ++o) {
            an[o] = 0.0;
            ad[o] = 0.0;
        }
        if (i < nx) {
            const int64_t m_lo = j0 - R > 0 ? j0 - R : 0;
            const int64_t m_hi = j0 + kColOut - 1 + R < ny - 1 ? j0 + kColOut - 1 + R : ny - 1;
            int64_t m = m_lo;
            // chunks of CH input rows: CH independent loads in flight and the 2 CH - 1 weights
            // they need in scalar registers, then CH x 16 fused multiply-adds
            constexpr int CH = HOLES ? 4 : 8;
            for (; m + CH - 1 <= m_hi; m += CH) {
                const double *w = gc + (m - j0 + R + 16);
                double wr[CH + kColOut - 1];
#pragma unroll
                for (int t = 0; t < CH + kColOut - 1; ++t) wr[t] = w[t - (kColOut - 1)];
                if (HOLES) {
                    double2 v[CH];
#pragma unroll
                    for (int q = 0; q < CH; ++q) v[q] = reinterpret_cast<const double2 *>(nd)[(m + q) * nx + i];
#pragma unroll
                    for (int q = 0; q < CH; ++q)
#pragma unroll
                        for (int o = 0; o < kColOut; ++o) {
                            an[o] = fma(wr[q - o + kColOut - 1], v[q].x, an[o]);
                            ad[o] = fma(wr[q - o + kColOut - 1], v[q].y, ad[o]);
                        }
                } else {
                    double v[CH];
#pragma unroll
                    for (int q = 0; q < CH; ++q) v[q] = nd[(m + q) * nx + i];
#pragma unroll
                    for (int q = 0; q < CH; ++q)
#pragma unroll
                        for (int o = 0; o < kColOut; ++o) an[o] = fma(wr[q - o + kColOut - 1], v[q], an[o]);
                }
            }
            for (; m <= m_hi; ++m) {
                const double *w = gc + (m - j0 + R + 16);
                if (HOLES) {
                    const double2 v = reinterpret_cast<const double2 *>(nd)[m * nx + i];
#pragma unroll
                    for (int o = 0; o < kColOut; ++o) {
                        an[o] = fma(w[-o], v.x, an[o]);
                        ad[o] = fma(w[-o], v.y, ad[o]);
                    }
                } else {
                    const double v = nd[m * nx + i];
#pragma unroll
                    for (int o = 0; o < kColOut; ++o) an[o] = fma(w[-o], v, an[o]);
                }
            }
#pragma unroll
            for (int o = 0; o < kColOut; ++o) {
                const int64_t j = j0 + o;
                if (j < ny) {
                    const int64_t k = j * nx + i;
                    const double h = (double)z[k];
                    const double lp = an[o] / (HOLES ? ad[o] : cx[i] * cy[j]);
                    out[k] = is_hit(h) ? (T)(mode == 0 ? lp : h - lp) : inf_of<T>();
                }
            }
        }
    }
}

int64_t grid_for(int64_t items) { return items < kMaxItems ? items : kMaxItems; }

}  // namespace

int launch_plane(const void *const *zin, void *const *zout, int n_maps, int64_t nx, int64_t ny,
                 int precision, int nb, double *part, double *coef, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double ci = 0.5 * (double)(nx - 1), cj = 0.5 * (double)(ny - 1);
    const dim3 g2((unsigned)nb, (unsigned)n_maps);
    if (precision == FSM_F64) {
        hipLaunchKernelGGL(plane_moments<double>, g2, dim3(256), 0, s, (const double *const *)zin, nx, ny, ci, cj, part);
        hipLaunchKernelGGL(plane_solve, dim3((unsigned)n_maps), dim3(256), 0, s, (const double *)part, nb, coef);
        hipLaunchKernelGGL(plane_apply<double>, g2, dim3(256), 0, s, (const double *const *)zin, (double *const *)zout, nx, ny, ci, cj, (const double *)coef);
    } else {
        hipLaunchKernelGGL(plane_moments<float>, g2, dim3(256), 0, s, (const float *const *)zin, nx, ny, ci, cj, part);
        hipLaunchKernelGGL(plane_solve, dim3((unsigned)n_maps), dim3(256), 0, s, (const double *)part, nb, coef);
        hipLaunchKernelGGL(plane_apply<float>, g2, dim3(256), 0, s, (const float *const *)zin, (float *const *)zout, nx, ny, ci, cj, (const double *)coef);
    }
    return (int)hipGetLastError();
}

int plane_blocks(int64_t ny, int n_maps)
{
    // about 2048 blocks over all maps, each at least a few rows when maps are many
    const int64_t want = std::max<int64_t>(8, std::min<int64_t>(kPlaneBlocks, 2048 / std::max(1, n_maps)));
    return (int)(ny < want ? ny : want);
}

size_t gauss_lds_bytes(int K8)
{
    const int L = kRowTile + K8 + 8;
    return sizeof(double) * (size_t)(L + (L >> 3) + 1);
}

int launch_scan_holes(const void *const *zin, int n_maps, int64_t n, int precision, int *flag, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    // about 8192 blocks over all maps, each striding over its map
    const int64_t blocks = (n + 255) / 256, per_map = std::max<int64_t>(1, 8192 / n_maps);
    const dim3 gr((unsigned)(blocks < per_map ? blocks : per_map), (unsigned)n_maps);
    hipLaunchKernelGGL(clear_flag, dim3(1), dim3(1), 0, s, flag);
    if (precision == FSM_F64)
        hipLaunchKernelGGL(scan_holes<double>, gr, dim3(256), 0, s, (const double *const *)zin, n, flag);
    else
        hipLaunchKernelGGL(scan_holes<float>, gr, dim3(256), 0, s, (const float *const *)zin, n, flag);
    return (int)hipGetLastError();
}

namespace {

template <typename T, bool HOLES>
void gauss_pair(const void *const *zin, void *const *zout, int n_maps, int64_t nx, int64_t ny, int R, int K8,
                const double *g_row, const double *g_col, const double *cx, const double *cy, void *nd, int mode,
                hipStream_t s)
{
    const int64_t row_items = ((nx + kRowTile - 1) / kRowTile) * ny;
    const int64_t col_items = ((nx + 63) / 64) * ((ny + kColRows - 1) / kColRows);
    const dim3 gr((unsigned)grid_for(row_items), (unsigned)n_maps);
    const dim3 gcol((unsigned)grid_for(col_items), (unsigned)n_maps);
    hipLaunchKernelGGL((gauss_rows<T, HOLES>), gr, dim3(kRowThreads), gauss_lds_bytes(K8), s,
                       (const T *const *)zin, nx, ny, R, K8, g_row, (double *)nd);
    hipLaunchKernelGGL((gauss_cols<T, HOLES>), gcol, dim3(64 * kColWaves), 0, s, (const T *const *)zin,
                       (T *const *)zout, nx, ny, R, g_col, cx, cy, (const double *)nd, mode);
}

}  // namespace

int launch_gauss(const void *const *zin, void *const *zout, int n_maps, int64_t nx, int64_t ny, int precision,
                 int R, int K8, const double *g_row, const double *g_col, const double *cx, const double *cy,
                 bool holes, void *nd, int mode, void *stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (precision == FSM_F64) {
        if (holes) gauss_pair<double, true>(zin, zout, n_maps, nx, ny, R, K8, g_row, g_col, cx, cy, nd, mode, s);
        else gauss_pair<double, false>(zin, zout, n_maps, nx, ny, R, K8, g_row, g_col, cx, cy, nd, mode, s);
    } else {
        if (holes) gauss_pair<float, true>(zin, zout, n_maps, nx, ny, R, K8, g_row, g_col, cx, cy, nd, mode, s);
        else gauss_pair<float, false>(zin, zout, n_maps, nx, ny, R, K8, g_row, g_col, cx, cy, nd, mode, s);
    }
    return (int)hipGetLastError();
}

}  // namespace fsm
