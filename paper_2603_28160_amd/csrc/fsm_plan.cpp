// fsm_plan.cpp -- host planner of libfsm: parameter validation, edge discretisation, the
// resolved tool path and the per-simulation tables the kernels read.
//
// Every quantity that needs a square root or a trigonometric function is computed here,
// once, in double precision with the C library, so the device kernels only add, subtract,
// multiply and divide.  The operation order of each expression is fixed (the build turns off
// contraction into fused multiply-adds), which makes the double-precision path reproduce the
// plain definition of the method bit for bit.
//
// The file also holds the host thread pool that builds large tables (and many plans) in
// parallel.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <limits>
#include <unistd.h>

#include "fsm_internal.h"

namespace fsm {
namespace {

// Worker threads that wait for jobs, so that a call does not pay for creating threads.
class HostPool {
public:
    HostPool() : pid_(getpid())
    {
        const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
        const int w = std::min(hw, 16) - 1;
        for (int i = 0; i < w; ++i) workers_.emplace_back([this] { loop(); });
    }
    bool run(int n, void (*f)(void *, int), void *ctx)
    {
        if (depth_ > 0 || workers_.empty() || getpid() != pid_) return false;
        std::unique_lock<std::mutex> busy(busy_, std::try_to_lock);
        if (!busy.owns_lock()) return false;
        {
            std::lock_guard<std::mutex> g(m_);
            f_ = f;
            ctx_ = ctx;
            n_ = n;
            next_.store(0);
            running_ = (int)workers_.size();
            ++gen_;
        }
        cv_.notify_all();
        ++depth_;
        work();
        --depth_;
        std::unique_lock<std::mutex> g(m_);
        done_.wait(g, [this] { return running_ == 0; });
        return true;
    }

private:
    static thread_local int depth_;   // > 0 inside a pool job (workers always)
    void work()
    {
        for (int k; (k = next_.fetch_add(1)) < n_;) f_(ctx_, k);
    }
    void loop()
    {
        depth_ = 1;
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> g(m_);
                cv_.wait(g, [&] { return gen_ != seen; });
                seen = gen_;
            }
            work();
            std::lock_guard<std::mutex> g(m_);
            if (--running_ == 0) done_.notify_one();
        }
    }
    const pid_t pid_;
    std::vector<std::thread> workers_;
    std::mutex m_, busy_;
    std::condition_variable cv_, done_;
    void (*f_)(void *, int) = nullptr;
    void *ctx_ = nullptr;
    int n_ = 0, running_ = 0;
    std::atomic<int> next_{0};
    uint64_t gen_ = 0;
};
thread_local int HostPool::depth_ = 0;

bool finite(double v) { return std::isfinite(v); }

// Angular position of tooth K on the cutter body: 2*pi*(K-1)/z_n of Eq. (3) with K counted
// from zero, or the variable pitch given by the caller.
double tooth_angle(const fsm_tool &t, int K)
{
    if (t.uniform_pitch) return ((2.0 * M_PI) * (double)K) / (double)t.n_teeth;
    return t.theta[K];
}

// Edge point p in the cutting-edge frame (x, 0, z).
//   round edge: Eq. (6) on the chord [-dL, dL]; the half chord is the larger of the depth-of
//     -cut chord sqrt(R^2 - (R - a_p)^2) and the feed criterion f_z / (2 cos gamma_f)
//     (Sec. 2.2), capped at R; the point sits on the circle z = R - sqrt(R^2 - l^2) (Eq. (1)).
//   ball end: sphere of radius D/2 about the tool axis, polar angle kappa from the tip to the
//     depth of cut plus the tilt.
void edge_point(const fsm_tool &t, const fsm_cut &c, int p, double &x, double &z)
{
    const int N = t.n_edge;
    if (t.kind == FSM_TOOL_ROUND) {
        const double R = t.R_edge;
        double half_ap = R;
        if (c.a_p < R) half_ap = std::sqrt(R * R - (R - c.a_p) * (R - c.a_p));
        const double half_fz = c.f_z / (2.0 * std::cos(t.rake_radial));
        double half = half_ap > half_fz ? half_ap : half_fz;
        if (half > R) half = R;
        double l = 0.0;
        if (N > 1) l = -half + ((2.0 * half) / (double)(N - 1)) * (double)p;
        x = l;
        z = R - std::sqrt(R * R - l * l);
    } else {
        const double Rb = t.D / 2.0;
        double u = 1.0 - c.a_p / Rb;
        if (u < 0.0) u = 0.0;
        double kmax = (std::fabs(t.tilt_lead) + std::fabs(t.tilt_side)) + std::acos(u);
        if (kmax > M_PI / 2.0) kmax = M_PI / 2.0;
        double k = 0.0;
        if (N > 1) k = (kmax * (double)p) / (double)(N - 1);
        x = Rb * std::sin(k);
        z = Rb * (1.0 - std::cos(k));
    }
}

int validate(const fsm_tool &t, const fsm_cut &c, const fsm_grid &g, std::string &err)
{
    auto bad = [&](const char *m) { err = m; return FSM_EINVAL; };
    if (t.kind != FSM_TOOL_ROUND && t.kind != FSM_TOOL_BALL) return bad("tool.kind must be 0 (round edge) or 1 (ball)");
    if (t.n_teeth < 1 || t.n_teeth > FSM_MAX_TEETH) return bad("tool.n_teeth must be in [1, 8]");
    if (t.n_edge < 1 || t.n_edge > FSM_MAX_EDGE) return bad("tool.n_edge must be in [1, 4096]");
    if (!finite(t.D) || !(t.D > 0.0)) return bad("tool.D must be finite and > 0");
    if (t.kind == FSM_TOOL_ROUND && (!finite(t.R_edge) || !(t.R_edge > 0.0)))
        return bad("tool.R_edge must be finite and > 0 for a round edge");
    const double angles[] = {t.helix, t.rake_radial, t.rake_axial, t.runout_phase, t.tilt_lead, t.tilt_side};
    for (double a : angles)
        if (!finite(a)) return bad("tool angles must be finite");
    if (!(std::fabs(t.helix) < M_PI / 2.0)) return bad("|tool.helix| must be < pi/2");
    if (!(std::fabs(t.rake_radial) < M_PI / 2.0)) return bad("|tool.rake_radial| must be < pi/2");
    if (!finite(t.runout_ecc) || t.runout_ecc < 0.0) return bad("tool.runout_ecc must be finite and >= 0");
    for (int k = 0; k < FSM_MAX_TEETH; ++k)
        if (!finite(t.theta[k]) || !finite(t.eps_r[k]) || !finite(t.eps_a[k]))
            return bad("tool.theta / eps_r / eps_a must be finite");
    if (!finite(c.f_z) || c.f_z < 0.0) return bad("cut.f_z must be finite and >= 0");
    if (!finite(c.a_p) || !(c.a_p > 0.0)) return bad("cut.a_p must be finite and > 0");
    if (!finite(c.a_e)) return bad("cut.a_e must be finite");
    if (!finite(c.phi0)) return bad("cut.phi0 must be finite");
    if (c.time_mode != FSM_TIME_PER_REV && c.time_mode != FSM_TIME_FIXED_DT) return bad("cut.time_mode unknown");
    if (c.time_mode == FSM_TIME_PER_REV && c.steps_per_rev < 1) return bad("cut.steps_per_rev must be >= 1");
    if (c.time_mode == FSM_TIME_FIXED_DT && (!finite(c.v_c) || !(c.v_c > 0.0) || !finite(c.dt) || !(c.dt > 0.0)))
        return bad("cut.v_c and cut.dt must be finite and > 0 in the fixed-time-step mode");
    if (std::isinf(c.x_end)) return bad("cut.x_end must be finite or NaN");
    if (c.n_passes < 0) return bad("cut.n_passes must be >= 0");
    if (c.n_steps < 0 || c.n_steps > (int64_t)INT32_MAX) return bad("cut.n_steps must be in [0, 2^31)");
    if (std::isinf(c.x_start) || std::isinf(c.y_first)) return bad("cut.x_start / y_first must be finite or NaN");
    if (!finite(g.x0) || !finite(g.y0)) return bad("grid origin must be finite");
    if (!finite(g.dd) || !(g.dd > 0.0)) return bad("grid.dd must be finite and > 0");
    if (g.nx < 1 || g.ny < 1) return bad("grid.nx and grid.ny must be >= 1");
    if (g.nx > (int64_t)INT32_MAX || g.ny > (int64_t)INT32_MAX || g.nx > INT64_MAX / g.ny)
        return bad("grid too large");
    return FSM_OK;
}

}  // namespace

bool pool_run(int n, void (*f)(void *, int), void *ctx)
{
    // never destroyed: its threads wait until the process ends, also in a forked child that
    // does not own them
    static HostPool *pool = new HostPool;
    return pool->run(n, f, ctx);
}

int build_plan(const fsm_tool &t, const fsm_cut &c, const fsm_grid &g, Plan &P,
               std::string &err, bool tables)
{
    int rc = validate(t, c, g, err);
    if (rc != FSM_OK) return rc;
    const int Z = t.n_teeth, N = t.n_edge;
    const bool fixed_dt = c.time_mode == FSM_TIME_FIXED_DT;
    P.kind = t.kind;
    P.z_n = Z;
    P.N = N;

    // --- edge points in the tool frame: Eq. (2), then the helix lag turn, then the
    // eccentric offset.  Each line is the matrix-vector product of that transformation
    // written out with its zero terms dropped (they only change the sign of a zero).
    P.pT.assign((size_t)Z * N * 3, 0.0);
    const double cf = std::cos(t.rake_radial), sf = std::sin(t.rake_radial);
    const double cp = std::cos(t.rake_axial), sp = std::sin(t.rake_axial);
    const double m02 = sf * sp, m12 = cf * sp;
    const double off = t.kind == FSM_TOOL_ROUND ? t.D / 2.0 : 0.0;
    const double tanb = std::tan(t.helix);
    const double rref = t.D / 2.0;
    // the edge profile and the helix lag depend on the point only, not on the tooth
    std::vector<double> el((size_t)N), ez((size_t)N), lc((size_t)N), ls((size_t)N);
    for (int p = 0; p < N; ++p) {
        edge_point(t, c, p, el[p], ez[p]);
        const double psi = (ez[p] * tanb) / rref;           // helix lag angle
        lc[p] = std::cos(psi);
        ls[p] = std::sin(psi);
    }
    for (int K = 0; K < Z; ++K) {
        const double tx = off + t.eps_r[K];
        const double ph = t.runout_phase + tooth_angle(t, K);
        const double ex = t.runout_ecc * std::cos(ph), ey = t.runout_ecc * std::sin(ph);
        for (int p = 0; p < N; ++p) {
            const double l = el[p], zc = ez[p];
            const double a0 = (cf * l + m02 * zc) + tx;     // Eq. (2), row 1
            const double a1 = (-sf) * l + m12 * zc;         // Eq. (2), row 2
            const double a2 = cp * zc + t.eps_a[K];         // Eq. (2), row 3
            const double cq = lc[p], sq = ls[p];
            const double b0 = cq * a0 + sq * a1;
            const double b1 = (-sq) * a0 + cq * a1;
            double *o = &P.pT[((size_t)K * N + p) * 3];
            o[0] = b0 + ex;
            o[1] = b1 + ey;
            o[2] = a2;
        }
    }

    // --- reach and the automatic path (feed along +X, passes along +Y)
    const double sl = std::fabs(std::sin(t.tilt_lead)), ss = std::fabs(std::sin(t.tilt_side));
    double reach = 0.0, pos_r = 0.0;
    for (size_t k = 0; k < (size_t)Z * N; ++k) {
        const double x = P.pT[3 * k], y = P.pT[3 * k + 1], z = P.pT[3 * k + 2];
        const double r = std::sqrt(x * x + y * y) + std::fabs(z) * (sl + ss);
        if (r > reach) reach = r;
        pos_r = std::max(pos_r, std::sqrt(x * x + y * y + z * z));
    }
    P.pos_r = pos_r;
    const double x_lo = g.x0 - 0.5 * g.dd, y_lo = g.y0 - 0.5 * g.dd;
    const double x_hi = x_lo + (double)g.nx * g.dd, y_hi = y_lo + (double)g.ny * g.dd;
    const double fpr = (double)Z * c.f_z;
    P.r_reach = reach;
    if (!(reach / g.dd < 536870912.0)) { err = "tool reach spans more than 2^29 cells"; return FSM_EINVAL; }
    P.x_start = std::isnan(c.x_start) ? x_lo - reach : c.x_start;
    const double x_end = std::isnan(c.x_end) ? x_hi + reach : c.x_end;
    // fixed-time-step mode (Sec. 4.3): spindle speed from the cutting speed, then the angular
    // and feed speeds; a step sits at time s dt
    const double n_rpm = fixed_dt ? (1000.0 * c.v_c) / (M_PI * t.D) : 0.0;
    const double omega = fixed_dt ? ((2.0 * M_PI) * n_rpm) / 60.0 : 0.0;
    const double v_f = fixed_dt ? (c.f_z * (double)Z * n_rpm) / 60.0 : 0.0;
    if (c.n_steps > 0) {
        P.n_steps = c.n_steps;
    } else if (fixed_dt) {
        double steps = v_f > 0.0 ? std::ceil(((x_end - P.x_start) / v_f) / c.dt) : 1.0;
        if (steps < 1.0) steps = 1.0;
        if (!(steps < (double)INT32_MAX)) { err = "path needs more than 2^31 steps per pass"; return FSM_EINVAL; }
        P.n_steps = (int64_t)steps;
    } else if (fpr > 0.0) {
        double revs = std::ceil((x_end - P.x_start) / fpr);
        if (revs < 1.0) revs = 1.0;
        if (!(revs * (double)c.steps_per_rev < (double)INT32_MAX)) { err = "path needs more than 2^31 steps per pass"; return FSM_EINVAL; }
        P.n_steps = (int64_t)revs * c.steps_per_rev;
    } else {
        P.n_steps = c.steps_per_rev;
    }
    // the angle table's period: a revolution, or every step of a pass in the fixed-step mode
    if (fixed_dt && (double)Z * (double)P.n_steps > (double)(1 << 26)) {
        err = "fixed-time-step angle table above 2^26 entries";
        return FSM_EINVAL;
    }
    const int S = fixed_dt ? (int)P.n_steps : c.steps_per_rev;
    P.S = S;
    if (c.n_passes > 0) {
        P.n_passes = c.n_passes;
    } else if (c.a_e > 0.0) {
        const double q = std::ceil(((y_hi + reach) - (y_lo - reach)) / c.a_e);
        if (!(q < 1e9)) { err = "path needs too many passes"; return FSM_EINVAL; }
        P.n_passes = (int64_t)q + 1;
    } else {
        P.n_passes = 1;
    }
    if (!std::isnan(c.y_first)) P.y_first = c.y_first;
    else if (c.a_e > 0.0) P.y_first = y_lo - reach;
    else P.y_first = g.y0 + 0.5 * (double)(g.ny - 1) * g.dd;
    if (P.n_passes > INT32_MAX / 2) { err = "too many passes"; return FSM_EINVAL; }
    const double evals = (double)P.n_passes * (double)P.n_steps * (double)Z * (double)N;
    if (!(evals < 4.0e18)) { err = "too many edge-point evaluations"; return FSM_EINVAL; }
    P.n_evals = P.n_passes * P.n_steps * Z * N;
    P.a_e = c.a_e;
    P.x_lo = x_lo;
    P.y_lo = y_lo;
    P.inv_dd = 1.0 / g.dd;
    P.nx = g.nx;
    P.ny = g.ny;
    P.tilt_lead = t.tilt_lead != 0.0;
    P.tilt_side = t.tilt_side != 0.0;
    P.tl_c = std::cos(t.tilt_lead);
    P.tl_s = std::sin(t.tilt_lead);
    P.ts_c = std::cos(t.tilt_side);
    P.ts_s = std::sin(t.tilt_side);
    P.n_groups = (N + kGroup - 1) / kGroup;
    P.x_hi = x_hi;
    P.y_hi = y_hi;
    if (!tables) return FSM_OK;

    // --- spindle angle of Eq. (3), alpha = phi + theta_K - omega t with omega t = 2 pi m / S,
    // m = step mod S: one (cos, sin) pair per tooth and step of a revolution.  Fixed-step
    // mode: omega t = omega (s dt) for every step s of a pass.
    // (large tables, as in the fixed-step mode, are filled in chunks on several threads)
    // a few thousand angles are cheaper on the calling thread than waking the pool
    constexpr int kChunk = 4096;          // angles per pool job
    constexpr int64_t kPoolAngles = 32768;
    P.cs.assign((size_t)Z * S * 2, 0.0);
    const int n_chunks = (int64_t)Z * S < kPoolAngles ? 1 : (S + kChunk - 1) / kChunk;
    const int chunk = (S + n_chunks - 1) / n_chunks;
    auto angles = [&](int job) {
        const int K = job / n_chunks, m0 = (job % n_chunks) * chunk;
        const int m1 = std::min(S, m0 + chunk);
        const double a = c.phi0 + tooth_angle(t, K);
        for (int m = m0; m < m1; ++m) {
            const double alpha = fixed_dt ? a - omega * ((double)m * c.dt)
                                          : a - ((2.0 * M_PI) * (double)m) / (double)S;
            P.cs[((size_t)K * S + m) * 2] = std::cos(alpha);
            P.cs[((size_t)K * S + m) * 2 + 1] = std::sin(alpha);
        }
    };
    if ((int64_t)Z * S < kPoolAngles) {
        for (int K = 0; K < Z; ++K) angles(K);
    } else {
        parallel_for(Z * n_chunks, angles);
    }
    // --- tool-centre x per step (Eq. (4) with the feed along X): z_n f_z per revolution, or
    // v_f (s dt) in the fixed-step mode; the kernels form it per step
    P.fixed_dt = fixed_dt;
    P.feed = fixed_dt ? v_f : fpr;
    P.dt = fixed_dt ? c.dt : 0.0;

    // --- culling radii.  Every point of a group stays within its distance rho from the
    // group's reference point under the rigid turn and tilts, so at any step the group's
    // points lie within rho of where the reference point lands.  The slack eps covers the
    // rounding of the test and of single-precision points.
    const double eps = 1e-5 * (reach + 1.0);
    P.gm.assign((size_t)Z * P.n_groups, 0.0);
    for (int K = 0; K < Z; ++K) {
        for (int gi = 0; gi < P.n_groups; ++gi) {
            const double *m = &P.pT[((size_t)K * N + group_ref(gi, N)) * 3];
            double rho = 0.0;
            for (int p = gi * kGroup; p < N && p < (gi + 1) * kGroup; ++p) {
                const double *q = &P.pT[((size_t)K * N + p) * 3];
                const double dx = q[0] - m[0], dy = q[1] - m[1], dz = q[2] - m[2];
                rho = std::max(rho, std::sqrt(dx * dx + dy * dy + dz * dz));
            }
            P.gm[(size_t)K * P.n_groups + gi] = rho + eps;
        }
    }
    P.cull_reach = reach + eps;
    return FSM_OK;
}

}  // namespace fsm
