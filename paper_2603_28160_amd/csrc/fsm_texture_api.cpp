// fsm_texture_api.cpp -- the C ABI of the surface-texture operators: F-operator (least-squares
// plane), areal Gaussian S- and L-filters and their chain with the roughness, applied to a
// Z-map in device memory (the measurement practice of Sec. 4.1.1).
//
// The host validates, computes the Gaussian weight tables, stages them with the map pointers
// in the context's workspace and turns the solved plane into mm units; every operation on the
// maps runs in fsm_texture.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fsm_runtime.h"
#include "fsm_spans.h"

using namespace fsm::rt;

namespace {

constexpr int kMaxHalfWidth = 3072;

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

bool valid_grid(const fsm_grid *g)
{
    return g && g->nx >= 1 && g->ny >= 1 && g->nx <= INT32_MAX && g->ny <= INT32_MAX &&
           g->nx <= INT64_MAX / g->ny / 16 && std::isfinite(g->x0) && std::isfinite(g->y0) &&
           std::isfinite(g->dd) && g->dd > 0.0;
}

int check_common(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zin, void *zout)
{
    if (!valid_grid(grid) || !zin || !zout || !valid_precision(precision))
        return set_err(ctx, FSM_EINVAL, "invalid grid, pointer or precision");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_err(ctx, e, "hipSetDevice");
    return FSM_OK;
}

// The maps of a call: an output shares no byte with another map's input or output, nor with
// its own input unless it is that input (in place); inputs may share bytes.
int check_maps(fsm_ctx *ctx, const fsm_grid *grid, int precision, int n, const void *const *zin,
               void *const *zout)
{
    const uintptr_t bytes = (uintptr_t)grid->nx * (uintptr_t)grid->ny *
                            (precision == FSM_F64 ? sizeof(double) : sizeof(float));
    std::vector<fsm::Span> spans;
    spans.reserve(2 * (size_t)n);
    for (int m = 0; m < n; ++m) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(zin[m]), b = reinterpret_cast<uintptr_t>(zout[m]);
        spans.push_back({b, b + bytes, m, false});
        if (a != b) spans.push_back({a, a + bytes, m, true});
    }
    const std::pair<int, int> o = fsm::first_conflict(std::move(spans));
    if (o.first < 0) return FSM_OK;
    if (o.first == o.second)
        return set_err(ctx, FSM_EINVAL, "map " + std::to_string(o.first) +
                                            ": output overlaps its input without being the same map");
    return set_err(ctx, FSM_EINVAL, "maps " + std::to_string(std::min(o.first, o.second)) + " and " +
                                        std::to_string(std::max(o.first, o.second)) +
                                        ": an output overlaps another map");
}

// Half-width in cells of the Gaussian window, or -1 when the request is invalid.
int half_width(const fsm_grid *g, double cutoff, double trunc)
{
    if (!(cutoff > 0.0) || !std::isfinite(cutoff) || !(trunc > 0.0) || !(trunc <= 4.0)) return -1;
    const double r = std::floor(trunc * cutoff / g->dd + 1e-9);
    if (!(r <= (double)kMaxHalfWidth)) return -1;
    return (int)r;
}

// Weight tables of one Gaussian filter in the staging region: row weights (K8), column
// weights (2R + 33, 16 zeros on either side), per-column and per-row sums of the weights whose
// cells lie inside the grid (nx, ny).  Offsets in doubles from the start of the region.
struct FilterTables {
    double cutoff = 0.0;
    int R = 0, K8 = 0, n_col = 0;
    size_t row = 0, col = 0, cx = 0, cy = 0, end = 0;
};

FilterTables plan_tables(const fsm_grid *g, double cutoff, int R, size_t at)
{
    FilterTables t;
    t.cutoff = cutoff;
    t.R = R;
    t.K8 = (2 * R + 1 + 7) / 8 * 8;
    t.n_col = 2 * R + 33;
    t.row = at;
    t.col = t.row + (size_t)t.K8;
    t.cx = t.col + (size_t)t.n_col;
    t.cy = t.cx + (size_t)g->nx;
    t.end = t.cy + (size_t)g->ny;
    return t;
}

void fill_tables(const fsm_grid *g, const FilterTables &t, double *h)
{
    std::memset(h + t.row, 0, sizeof(double) * (t.end - t.row));
    // w(a) = exp(-pi (a dd / (alpha cutoff))^2), a = k - R
    const double alpha = std::sqrt(std::log(2.0) / M_PI);
    const int R = t.R;
    std::vector<double> prefix((size_t)2 * R + 2, 0.0);
    for (int k = 0; k <= 2 * R; ++k) {
        const double u = ((double)(k - R) * g->dd) / (alpha * t.cutoff);
        const double w = std::exp(-M_PI * (u * u));
        h[t.row + (size_t)k] = w;
        h[t.col + 16 + (size_t)k] = w;
        prefix[(size_t)k + 1] = prefix[(size_t)k] + w;
    }
    // sum of the weights whose offset keeps index i + a inside [0, n)
    auto in_grid_sum = [&](int64_t i, int64_t n) {
        const int64_t lo = std::max<int64_t>(0, R - i), hi = std::min<int64_t>(2 * R, R + (n - 1 - i));
        return prefix[(size_t)hi + 1] - prefix[(size_t)lo];
    };
    for (int64_t i = 0; i < g->nx; ++i) h[t.cx + (size_t)i] = in_grid_sum(i, g->nx);
    for (int64_t j = 0; j < g->ny; ++j) h[t.cy + (size_t)j] = in_grid_sum(j, g->ny);
}

// One pass through the texture operators on `stream` over n maps of one grid: up to two
// filters (the first smoothing, the second keeping the roughness part), with a least-squares
// plane removed between them.  zin/zout: host arrays of n device map pointers.
struct Chain {
    int n_filters = 0;
    FilterTables f[2];
    int mode[2] = {FSM_FILTER_SMOOTH, FSM_FILTER_ROUGH};
    bool level = false;
};

constexpr size_t kScratchBudget = (size_t)4 << 30;   // bytes of filter scratch per group of maps

int run_chain(fsm_ctx *ctx, const fsm_grid *grid, int precision, int n, const void *const *zin,
              void *const *zout, const Chain &c, double *planes, hipStream_t s)
{
    const int64_t nx = grid->nx, ny = grid->ny;
    for (int k = 0; k < c.n_filters; ++k)
        if (fsm::gauss_lds_bytes(c.f[k].K8) > ctx->max_lds)
            return set_err(ctx, FSM_EINVAL, "filter window too wide for the device's LDS");
    const size_t per_map = c.n_filters ? (size_t)16 * (size_t)nx * (size_t)ny : 0;
    // maps of a group share the launches (one grid row per map: at most 65535)
    int group = per_map ? (int)std::max<size_t>(1, std::min<size_t>((size_t)n, kScratchBudget / per_map)) : n;
    group = std::min(group, 65535);
    const int nb = fsm::plane_blocks(ny, group);
    // device: [weight tables][input and output pointer arrays][plane partials][plane
    // coefficients, 4 per map][hole flag][filter scratch of one group]
    const size_t n_w = c.n_filters ? c.f[c.n_filters - 1].end : 0;
    const size_t ptr_at = align256(sizeof(double) * n_w);
    const size_t part_at = ptr_at + align256(sizeof(void *) * 2 * (size_t)n);
    const size_t coef_at = part_at + align256(sizeof(double) * 9 * (size_t)nb * (size_t)group);
    const size_t flag_at = coef_at + align256(sizeof(double) * 4 * (size_t)n);
    const size_t nd_at = flag_at + 256;
    // host staging: the same first two parts, then the coefficients and the flag read back
    const size_t h_coef_at = part_at;
    const size_t h_flag_at = h_coef_at + align256(sizeof(double) * 4 * (size_t)n);
    int rc = ensure(ctx, ctx->ws, nd_at + per_map * (size_t)group, h_flag_at + 64, 1);
    if (rc != FSM_OK) return rc;
    char *dev = static_cast<char *>(ctx->ws.d_ws);
    char *host = static_cast<char *>(ctx->ws.h_ws);
    double *h_coef = reinterpret_cast<double *>(host + h_coef_at);
    int *h_flag = reinterpret_cast<int *>(host + h_flag_at);
    double *d_coef = reinterpret_cast<double *>(dev + coef_at);
    int *d_flag = reinterpret_cast<int *>(dev + flag_at);
    // no earlier copy from the staging is in flight: every call here waits for its stream
    for (int k = 0; k < c.n_filters; ++k) fill_tables(grid, c.f[k], reinterpret_cast<double *>(host));
    void **h_ptr = reinterpret_cast<void **>(host + ptr_at);
    for (int m = 0; m < n; ++m) {
        h_ptr[m] = const_cast<void *>(zin[m]);
        h_ptr[n + m] = zout[m];
    }
    hipError_t e = hipMemcpyAsync(dev, host, part_at, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(tables)");
    const void *const *d_in = reinterpret_cast<const void *const *>(dev + ptr_at);
    void *const *d_out = reinterpret_cast<void *const *>(dev + ptr_at) + n;
    bool holes = true;
    if (c.n_filters) {
        // filters and the plane keep the set of empty cells, so one scan serves the chain
        for (int m0 = 0; m0 < n; m0 += 65535) {
            const int cnt = std::min(65535, n - m0);
            int he = fsm::launch_scan_holes(d_in + m0, cnt, nx * ny, precision, d_flag, s);
            if (he) return hip_err(ctx, (hipError_t)he, "hole scan");
            e = hipMemcpyAsync(h_flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(flag)");
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
            holes = *h_flag != 0;
            if (holes) break;
        }
    }
    const double *w = reinterpret_cast<const double *>(dev);
    for (int m0 = 0; m0 < n; m0 += group) {
        const int cnt = std::min(group, n - m0);
        const void *const *cur = d_in + m0;
        void *const *dst = d_out + m0;
        auto filter = [&](int k) {
            const FilterTables &t = c.f[k];
            int he = fsm::launch_gauss(cur, dst, cnt, nx, ny, precision, t.R, t.K8, w + t.row, w + t.col,
                                       w + t.cx, w + t.cy, holes, dev + nd_at, c.mode[k], s);
            cur = dst;
            return he ? hip_err(ctx, (hipError_t)he, "filter kernels") : FSM_OK;
        };
        int k = 0;
        if (c.level && c.n_filters == 2) {
            rc = filter(k++);
            if (rc != FSM_OK) return rc;
        }
        if (c.level) {
            int he = fsm::launch_plane(cur, dst, cnt, nx, ny, precision, nb,
                                       reinterpret_cast<double *>(dev + part_at), d_coef + 4 * (size_t)m0, s);
            if (he) return hip_err(ctx, (hipError_t)he, "plane kernels");
            cur = dst;
        }
        for (; k < c.n_filters; ++k) {
            rc = filter(k);
            if (rc != FSM_OK) return rc;
        }
        if (cur != dst) {
            // nothing switched on: the outputs take the inputs
            const size_t bytes = (size_t)nx * (size_t)ny * (precision == FSM_F64 ? sizeof(double) : sizeof(float));
            for (int m = m0; m < m0 + cnt; ++m) {
                if (zout[m] == zin[m]) continue;
                e = hipMemcpyAsync(zout[m], zin[m], bytes, hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(copy)");
            }
        }
    }
    if (c.level) {
        e = hipMemcpyAsync(h_coef, d_coef, sizeof(double) * 4 * (size_t)n, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(plane)");
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
    // z = c0 + cu u + cv v with u = (x - x0)/dd - ci, v = (y - y0)/dd - cj
    const double ci = 0.5 * (double)(nx - 1), cj = 0.5 * (double)(ny - 1);
    for (int m = 0; m < n; ++m) {
        double pl[3] = {0.0, 0.0, 0.0};
        if (c.level) {
            const double *q = h_coef + 4 * (size_t)m;
            if (q[3] == 0.0)
                return set_err(ctx, FSM_EINVAL, "map " + std::to_string(m) +
                                                ": fewer than three hit cells, or all on one line");
            pl[0] = q[0] - q[1] * (grid->x0 / grid->dd + ci) - q[2] * (grid->y0 / grid->dd + cj);
            pl[1] = q[1] / grid->dd;
            pl[2] = q[2] / grid->dd;
        }
        if (planes) std::memcpy(planes + 3 * (size_t)m, pl, sizeof(pl));
    }
    return FSM_OK;
}

// The chain of a texture specification: S-filter, plane, L-filter, each when switched on.
int chain_of(fsm_ctx *ctx, const fsm_grid *grid, const fsm_texture_spec *spec, Chain &c, bool &split)
{
    if (!spec || !(spec->lambda_s >= 0.0) || !(spec->lambda_c >= 0.0) ||
        !std::isfinite(spec->lambda_s) || !std::isfinite(spec->lambda_c))
        return set_err(ctx, FSM_EINVAL, "invalid texture specification");
    c.level = spec->level != 0;
    const double cut[2] = {spec->lambda_s, spec->lambda_c};
    const int modes[2] = {FSM_FILTER_SMOOTH, FSM_FILTER_ROUGH};
    size_t at = 0;
    for (int k = 0; k < 2; ++k) {
        if (!(cut[k] > 0.0)) continue;
        const int R = half_width(grid, cut[k], spec->trunc);
        if (R < 0) return set_err(ctx, FSM_EINVAL, "cut-off must be > 0, trunc in (0, 4], half-width <= 3072 cells");
        c.f[c.n_filters] = plan_tables(grid, cut[k], R, at);
        c.mode[c.n_filters] = modes[k];
        at = c.f[c.n_filters].end;
        ++c.n_filters;
    }
    // run_chain removes the plane after a first of two filters, else before its filter: an
    // S-filter alone with the plane needs two runs
    split = c.level && c.n_filters == 1 && c.mode[0] == FSM_FILTER_SMOOTH;
    return FSM_OK;
}

int texture_maps(fsm_ctx *ctx, const fsm_grid *grid, int precision, int n, const void *const *zin,
                 void *const *zout, const fsm_texture_spec *spec, fsm_rough *out, double *planes,
                 hipStream_t s)
{
    Chain c;
    bool split = false;
    int rc = chain_of(ctx, grid, spec, c, split);
    if (rc != FSM_OK) return rc;
    if (split) {
        Chain s1;
        s1.n_filters = 1;
        s1.f[0] = c.f[0];
        s1.mode[0] = FSM_FILTER_SMOOTH;
        rc = run_chain(ctx, grid, precision, n, zin, zout, s1, nullptr, s);
        if (rc != FSM_OK) return rc;
        Chain f;
        f.level = true;
        rc = run_chain(ctx, grid, precision, n, zout, zout, f, planes, s);
    } else {
        rc = run_chain(ctx, grid, precision, n, zin, zout, c, planes, s);
    }
    if (rc != FSM_OK) return rc;
    std::vector<void *> maps(zout, zout + n);
    return roughness_maps(ctx, grid, precision, maps, out, s);
}

}  // namespace

extern "C" {

int fsm_level(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zmap_in,
              void *zmap_out, double plane[3], void *stream)
{
    if (!ctx) return FSM_EINVAL;
    try {
        int rc = check_common(ctx, grid, precision, zmap_in, zmap_out);
        if (rc == FSM_OK) rc = check_maps(ctx, grid, precision, 1, &zmap_in, &zmap_out);
        if (rc != FSM_OK) return rc;
        Chain c;
        c.level = true;
        return run_chain(ctx, grid, precision, 1, &zmap_in, &zmap_out, c, plane, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

int fsm_filter(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zmap_in,
               void *zmap_out, double cutoff, double trunc, int mode, void *stream)
{
    if (!ctx) return FSM_EINVAL;
    try {
        int rc = check_common(ctx, grid, precision, zmap_in, zmap_out);
        if (rc == FSM_OK) rc = check_maps(ctx, grid, precision, 1, &zmap_in, &zmap_out);
        if (rc != FSM_OK) return rc;
        if (mode != FSM_FILTER_SMOOTH && mode != FSM_FILTER_ROUGH)
            return set_err(ctx, FSM_EINVAL, "unknown filter mode");
        const int R = half_width(grid, cutoff, trunc);
        if (R < 0) return set_err(ctx, FSM_EINVAL, "cut-off must be > 0, trunc in (0, 4], half-width <= 3072 cells");
        Chain c;
        c.n_filters = 1;
        c.f[0] = plan_tables(grid, cutoff, R, 0);
        c.mode[0] = mode;
        return run_chain(ctx, grid, precision, 1, &zmap_in, &zmap_out, c, nullptr, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

int fsm_texture(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zmap_in,
                void *zmap_out, const fsm_texture_spec *spec, fsm_rough *out, double plane[3],
                void *stream)
{
    if (!ctx) return FSM_EINVAL;
    try {
        int rc = check_common(ctx, grid, precision, zmap_in, zmap_out);
        if (rc == FSM_OK) rc = check_maps(ctx, grid, precision, 1, &zmap_in, &zmap_out);
        if (rc != FSM_OK) return rc;
        if (!out) return set_err(ctx, FSM_EINVAL, "no result record");
        return texture_maps(ctx, grid, precision, 1, &zmap_in, &zmap_out, spec, out, plane,
                            static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

int fsm_texture_batch(fsm_ctx *ctx, int n, const fsm_grid *grid, int precision,
                      const void *const *zmaps_in, void *const *zmaps_out,
                      const fsm_texture_spec *spec, fsm_rough *out, double *planes, void *stream)
{
    if (!ctx) return FSM_EINVAL;
    try {
        if (n < 0 || (n > 0 && (!zmaps_in || !zmaps_out || !out)))
            return set_err(ctx, FSM_EINVAL, "invalid map count or arrays");
        if (n == 0) return FSM_OK;
        for (int m = 0; m < n; ++m) {
            int rc = check_common(ctx, grid, precision, zmaps_in[m], zmaps_out[m]);
            if (rc != FSM_OK) return rc;
        }
        int rc = check_maps(ctx, grid, precision, n, zmaps_in, zmaps_out);
        if (rc != FSM_OK) return rc;
        return texture_maps(ctx, grid, precision, n, zmaps_in, zmaps_out, spec, out, planes,
                            static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

}  // extern "C"
