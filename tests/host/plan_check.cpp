// Host check of the planner (build_plan) for the sanitizers: a ball end with lead tilt, a
// round-edge face mill with variable pitch, per-insert offsets, rake, runout and both tilts,
// the paper's fixed time step (its angle table filled on the thread pool), and a one-point
// edge.  Every plan's tables have the sizes the planner states, hold finite values, and the
// same plan built twice is identical.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "fsm_internal.h"

static int fail(const char *what)
{
    std::printf("FAIL %s\n", what);
    return 1;
}

static bool same(const fsm::Plan &a, const fsm::Plan &b)
{
    return a.pT == b.pT && a.cs == b.cs && a.gm == b.gm && a.n_steps == b.n_steps &&
           a.n_passes == b.n_passes && a.r_reach == b.r_reach;
}

static int check(const fsm_tool &t, const fsm_cut &c, const fsm_grid &g, const char *name)
{
    std::string err;
    fsm::Plan p, q;
    if (fsm::build_plan(t, c, g, p, err, true) != FSM_OK) {
        std::printf("%s: %s\n", name, err.c_str());
        return fail(name);
    }
    if (fsm::build_plan(t, c, g, q, err, true) != FSM_OK || !same(p, q)) return fail(name);
    if (p.pT.size() != (size_t)p.z_n * p.N * 3 || p.cs.size() != (size_t)p.z_n * p.S * 2 ||
        p.gm.size() != (size_t)p.z_n * p.n_groups)
        return fail(name);
    for (double v : p.pT)
        if (!std::isfinite(v)) return fail(name);
    for (double v : p.cs)
        if (!(std::fabs(v) <= 1.0)) return fail(name);
    for (double v : p.gm)
        if (!(v >= 0.0 && std::isfinite(v))) return fail(name);
    return 0;
}

int main()
{
    fsm_grid g = {-2.4995, -2.4995, 0.001, 500, 400};
    fsm_tool ball;
    std::memset(&ball, 0, sizeof ball);
    ball.kind = FSM_TOOL_BALL;
    ball.n_teeth = 4;
    ball.n_edge = 64;
    ball.uniform_pitch = 1;
    ball.D = 6.0;
    ball.helix = 30 * M_PI / 180;
    ball.runout_ecc = 0.004;
    ball.runout_phase = 1.0;
    ball.tilt_lead = 15 * M_PI / 180;
    fsm_cut cut;
    std::memset(&cut, 0, sizeof cut);
    cut.f_z = 0.08;
    cut.a_p = 0.5;
    cut.a_e = 0.3;
    cut.steps_per_rev = 720;
    cut.x_start = cut.y_first = cut.x_end = NAN;
    if (check(ball, cut, g, "ball")) return 1;

    fsm_tool face = ball;
    face.kind = FSM_TOOL_ROUND;
    face.n_teeth = 5;
    face.n_edge = 30;
    face.uniform_pitch = 0;
    face.D = 40.0;
    face.R_edge = 6.0;
    face.helix = 0.0;
    face.rake_radial = 0.1;
    face.rake_axial = -0.05;
    face.tilt_side = -0.12;
    for (int K = 0; K < 5; ++K) {
        face.theta[K] = 1.2 * K + 0.05 * K * K;
        face.eps_r[K] = -0.026 * K;
        face.eps_a[K] = 0.009 * K;
    }
    fsm_cut fc = cut;
    fc.f_z = 0.4;
    fc.a_p = 0.4;
    fc.a_e = 4.0;
    fc.steps_per_rev = 500;
    if (check(face, fc, g, "face")) return 1;

    // the paper's fixed time step: one angle per step and tooth over the whole travel
    fsm_cut fixed = fc;
    fixed.time_mode = FSM_TIME_FIXED_DT;
    fixed.v_c = 200.0;
    fixed.dt = 4e-7;
    fixed.x_start = -5.0;
    fixed.x_end = 5.0;
    fixed.n_passes = 1;
    fixed.y_first = 0.0;
    if (check(face, fixed, g, "fixed time step")) return 1;

    fsm_tool one = ball;
    one.n_edge = 1;
    one.n_teeth = 1;
    if (check(one, cut, g, "one point")) return 1;
    std::printf("OK\n");
    return 0;
}
