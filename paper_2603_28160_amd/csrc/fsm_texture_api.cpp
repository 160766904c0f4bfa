// fsm_texture_api.cpp -- the C ABI of the surface-texture operators: F-operator (least-squares
// plane), areal Gaussian S- and L-filters and their chain with the roughness, applied to a
// Z-map in device memory (the measurement practice of Sec. 4.1.1).
//
// The host only validates, computes the Gaussian weight tables and stages them in the
// context's workspace; every operation on the map runs in fsm_texture.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fsm_runtime.h"

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

// Half-width in cells of the Gaussian window, or -1 when the request is invalid.
int half_width(const fsm_grid *g, double cutoff, double trunc)
{
    if (!(cutoff > 0.0) || !std::isfinite(cutoff) || !(trunc > 0.0) || !(trunc <= 4.0)) return -1;
    const double r = std::floor(trunc * cutoff / g->dd + 1e-9);
    if (!(r <= (double)kMaxHalfWidth)) return -1;
    return (int)r;
}

int do_level(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zin, void *zout,
             double plane[3], hipStream_t s)
{
    const size_t coef_at = align256(sizeof(double) * fsm::kPlanePartials);
    int rc = ensure(ctx, ctx->ws, coef_at + 256, 256, 1);
    if (rc != FSM_OK) return rc;
    char *dev = static_cast<char *>(ctx->ws.d_ws);
    double *coef = reinterpret_cast<double *>(dev + coef_at);
    int he = fsm::launch_plane(zin, zout, grid->nx, grid->ny, precision,
                               reinterpret_cast<double *>(dev), coef, s);
    if (he) return hip_err(ctx, (hipError_t)he, "plane kernels");
    double *h = static_cast<double *>(ctx->ws.h_ws);
    hipError_t e = hipMemcpyAsync(h, coef, 4 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(plane)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
    if (h[3] == 0.0)
        return set_err(ctx, FSM_EINVAL, "fewer than three hit cells, or all on one line");
    if (plane) {
        // z = c0 + cu u + cv v with u = (x - x0)/dd - ci, v = (y - y0)/dd - cj
        const double ci = 0.5 * (double)(grid->nx - 1), cj = 0.5 * (double)(grid->ny - 1);
        const double bx = h[1] / grid->dd, by = h[2] / grid->dd;
        plane[0] = h[0] - h[1] * (grid->x0 / grid->dd + ci) - h[2] * (grid->y0 / grid->dd + cj);
        plane[1] = bx;
        plane[2] = by;
    }
    return FSM_OK;
}

// One Gaussian filter pass: stage the weight tables, find out whether the map has empty cells
// (the hole-free kernels sum only numerators), then the row and column passes.
int filter_once(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zin, void *zout,
                double cutoff, double trunc, int mode, hipStream_t s)
{
    const int R = half_width(grid, cutoff, trunc);
    if (R < 0) return set_err(ctx, FSM_EINVAL, "cut-off must be > 0, trunc in (0, 4], half-width <= 3072 cells");
    const int K8 = (2 * R + 1 + 7) / 8 * 8;
    const int n_col = 2 * R + 33;
    if (fsm::gauss_lds_bytes(K8) > ctx->max_lds)
        return set_err(ctx, FSM_EINVAL, "filter window too wide for the device's LDS");
    const int64_t nx = grid->nx, ny = grid->ny;
    // staging: row weights, column weights, per-column and per-row in-grid weight sums
    const size_t n_w = (size_t)K8 + (size_t)n_col + (size_t)nx + (size_t)ny;
    const size_t w_bytes = sizeof(double) * n_w;
    const size_t flag_at = align256(w_bytes);
    const size_t nd_at = flag_at + 256;
    const size_t nd_bytes = (size_t)16 * (size_t)nx * (size_t)ny;
    int rc = ensure(ctx, ctx->ws, nd_at + nd_bytes, w_bytes + 64, 1);
    if (rc != FSM_OK) return rc;
    // no earlier copy from the staging is in flight: every call here waits for its stream
    double *h = static_cast<double *>(ctx->ws.h_ws);
    std::memset(h, 0, w_bytes);
    // w(a) = exp(-pi (a dd / (alpha cutoff))^2), a = k - R
    const double alpha = std::sqrt(std::log(2.0) / M_PI);
    std::vector<double> prefix((size_t)2 * R + 2, 0.0);
    for (int k = 0; k <= 2 * R; ++k) {
        const double u = ((double)(k - R) * grid->dd) / (alpha * cutoff);
        const double w = std::exp(-M_PI * (u * u));
        h[k] = w;                         // row table
        h[K8 + 16 + k] = w;               // column table
        prefix[(size_t)k + 1] = prefix[(size_t)k] + w;
    }
    // sum of the weights whose offset keeps index t + a inside [0, n)
    auto in_grid_sum = [&](int64_t t, int64_t n) {
        const int64_t lo = std::max<int64_t>(0, R - t), hi = std::min<int64_t>(2 * R, R + (n - 1 - t));
        return prefix[(size_t)hi + 1] - prefix[(size_t)lo];
    };
    double *cx = h + K8 + n_col, *cy = cx + nx;
    for (int64_t i = 0; i < nx; ++i) cx[i] = in_grid_sum(i, nx);
    for (int64_t j = 0; j < ny; ++j) cy[j] = in_grid_sum(j, ny);
    char *dev = static_cast<char *>(ctx->ws.d_ws);
    hipError_t e = hipMemcpyAsync(dev, h, w_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(weights)");
    int *d_flag = reinterpret_cast<int *>(dev + flag_at);
    int he = fsm::launch_scan_holes(zin, nx * ny, precision, d_flag, s);
    if (he) return hip_err(ctx, (hipError_t)he, "hole scan");
    int *h_flag = reinterpret_cast<int *>(h + n_w);
    e = hipMemcpyAsync(h_flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(flag)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
    const double *g_row = reinterpret_cast<const double *>(dev);
    const double *g_col = g_row + K8;
    he = fsm::launch_gauss(zin, zout, nx, ny, precision, R, K8, g_row, g_col, g_col + n_col,
                           g_col + n_col + nx, *h_flag != 0, dev + nd_at, mode, s);
    if (he) return hip_err(ctx, (hipError_t)he, "filter kernels");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(ctx, e, "hipStreamSynchronize");
    return FSM_OK;
}

}  // namespace

extern "C" {

int fsm_level(fsm_ctx *ctx, const fsm_grid *grid, int precision, const void *zmap_in,
              void *zmap_out, double plane[3], void *stream)
{
    if (!ctx) return FSM_EINVAL;
    try {
        int rc = check_common(ctx, grid, precision, zmap_in, zmap_out);
        if (rc != FSM_OK) return rc;
        return do_level(ctx, grid, precision, zmap_in, zmap_out, plane, static_cast<hipStream_t>(stream));
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
        if (rc != FSM_OK) return rc;
        if (mode != FSM_FILTER_SMOOTH && mode != FSM_FILTER_ROUGH)
            return set_err(ctx, FSM_EINVAL, "unknown filter mode");
        return filter_once(ctx, grid, precision, zmap_in, zmap_out, cutoff, trunc, mode,
                           static_cast<hipStream_t>(stream));
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
        if (rc != FSM_OK) return rc;
        if (!spec || !out || !(spec->lambda_s >= 0.0) || !(spec->lambda_c >= 0.0) ||
            !std::isfinite(spec->lambda_s) || !std::isfinite(spec->lambda_c))
            return set_err(ctx, FSM_EINVAL, "invalid texture specification");
        if ((spec->lambda_s > 0.0 && half_width(grid, spec->lambda_s, spec->trunc) < 0) ||
            (spec->lambda_c > 0.0 && half_width(grid, spec->lambda_c, spec->trunc) < 0))
            return set_err(ctx, FSM_EINVAL, "cut-off must be > 0, trunc in (0, 4], half-width <= 3072 cells");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const void *cur = zmap_in;
        if (spec->lambda_s > 0.0) {
            rc = filter_once(ctx, grid, precision, cur, zmap_out, spec->lambda_s, spec->trunc,
                             FSM_FILTER_SMOOTH, s);
            if (rc != FSM_OK) return rc;
            cur = zmap_out;
        }
        double pl[3] = {0.0, 0.0, 0.0};
        if (spec->level) {
            rc = do_level(ctx, grid, precision, cur, zmap_out, pl, s);
            if (rc != FSM_OK) return rc;
            cur = zmap_out;
        }
        if (spec->lambda_c > 0.0) {
            rc = filter_once(ctx, grid, precision, cur, zmap_out, spec->lambda_c, spec->trunc,
                             FSM_FILTER_ROUGH, s);
            if (rc != FSM_OK) return rc;
            cur = zmap_out;
        }
        if (cur != zmap_out) {
            const size_t bytes = (size_t)grid->nx * (size_t)grid->ny *
                                 (precision == FSM_F64 ? sizeof(double) : sizeof(float));
            hipError_t e = hipMemcpyAsync(zmap_out, cur, bytes, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_err(ctx, e, "hipMemcpyAsync(copy)");
        }
        if (plane) std::memcpy(plane, pl, sizeof(pl));
        return fsm_roughness(ctx, grid, precision, zmap_out, out, stream);
    } catch (const std::bad_alloc &) {
        return set_err(ctx, FSM_ENOMEM, "host allocation failed");
    } catch (...) {
        return set_err(ctx, FSM_EINVAL, "unexpected host exception");
    }
}

}  // extern "C"
