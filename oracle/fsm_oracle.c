/*
 * fsm_oracle.c -- FP64 CPU oracle for the forward solution method (FSM) of milled surface
 * topography.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, obviously correct restatement of the method that
 * the GPU library is checked against.  It shares no code with the library.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * The method (Sec. 2): discretise the cutting edge into points (Eq. (1), (6)); carry every
 * point through the chain of homogeneous transformations cutting edge -> tool -> spindle ->
 * workpiece (Eq. (2)-(5)) at every time step; bin each workpiece-frame point into the
 * sampling boundary of a grid node (Eq. (7)) and keep the lowest height per node (Sec. 2.3).
 * The loops run in the order of the method's flowchart: pass, time step, tooth, edge point.
 *
 * Each transformation is a 4x4 homogeneous matrix applied to the point with a plain
 * matrix-vector product, term by term from left to right (no fused multiply-add; build with
 * -ffp-contract=off -fno-builtin).  Extensions beyond the paper's face-milling geometry, each
 * one an extra matrix in the chain that is the identity when its parameter is zero:
 *   - helix: trailing rotation about the tool axis by psi = z_prof * tan(beta) / (D/2);
 *   - eccentric runout: translation (e cos lambda, e sin lambda, 0) in the cutter-body
 *     frame, i.e. phase lambda + theta_K in the frame of tooth K;
 *   - tilt: rotation about workpiece Y by tilt_lead, then about X by tilt_side;
 *   - ball end: a sphere of radius D/2 on the tool axis replaces the circular insert.
 * Feed runs along +X and parallel passes step along +Y.
 *
 * Parity status: positions pinned by closed forms (special angles, rigid-motion invariants,
 * helix lag angle, sphere lowest point); binning and per-cell minimum pinned by brute force on
 * tiny grids; feed-mark and scallop heights pinned by their closed forms; roughness pinned by
 * closed-form surfaces; the time discretisation pinned by the trajectory-point counts of the
 * paper's performance table.
 */
#include "fsm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double m4[4][4];

/* r = M v, summed left to right. */
static void mv(const m4 M, const double v[4], double r[4])
{
    for (int i = 0; i < 4; ++i)
        r[i] = ((M[i][0] * v[0] + M[i][1] * v[1]) + M[i][2] * v[2]) + M[i][3] * v[3];
}

static void m_identity(m4 M)
{
    memset(M, 0, sizeof(m4));
    M[0][0] = M[1][1] = M[2][2] = M[3][3] = 1.0;
}

static int check_tool(const or_tool *t)
{
    if (!t) return -1;
    if (t->kind != 0 && t->kind != 1) return -1;
    if (t->n_teeth < 1 || t->n_teeth > OR_MAX_TEETH || t->n_edge < 1) return -1;
    if (!(t->D > 0.0)) return -1;
    if (t->kind == 0 && !(t->R_edge > 0.0)) return -1;
    return 0;
}

static int check_cut(const or_cut *c)
{
    if (!c) return -1;
    if (!(c->f_z >= 0.0) || !(c->a_p > 0.0)) return -1;
    if (c->n_passes < 0 || c->n_steps < 0) return -1;
    if (c->time_mode == 0) return c->S < 1 ? -1 : 0;
    if (c->time_mode == 1) return (c->v_c > 0.0 && c->dt > 0.0) ? 0 : -1;
    return -1;
}

/* Fixed-time-step mode (the paper's own time discretisation, Sec. 4.3): spindle speed
 * n = 1000 v_c / (pi D) rev/min from the cutting speed, angular speed omega = 2 pi n / 60,
 * feed speed v_f = f_z z_n n / 60 (mm/s); step s sits at time t = s dt. */
static double spindle_rpm(const or_tool *t, const or_cut *c) { return (1000.0 * c->v_c) / (M_PI * t->D); }
static double omega_of(const or_tool *t, const or_cut *c) { return ((2.0 * M_PI) * spindle_rpm(t, c)) / 60.0; }
static double feed_speed(const or_tool *t, const or_cut *c)
{
    return (c->f_z * (double)t->n_teeth * spindle_rpm(t, c)) / 60.0;
}

static int check_grid(const or_grid *g)
{
    if (!g || !(g->dd > 0.0) || g->nx < 1 || g->ny < 1) return -1;
    return 0;
}

/* Angular position of tooth K on the cutter body: 2*pi*(K-1)/z_n of Eq. (3) (K counted from
 * zero here), or the given variable pitch. */
static double tooth_angle(const or_tool *t, int K)
{
    if (t->uniform_pitch) return ((2.0 * M_PI) * (double)K) / (double)t->n_teeth;
    return t->theta[K];
}

/* ---- edge discretisation ---------------------------------------------------------------- */

/* Point p of the discretised edge in the cutting-edge frame, and the profile height used for
 * the helix lag.  Round edge: Eq. (6) with the chord rule of Sec. 2.2 (z_C read as a_p, the
 * half chord capped at R).  Ball end: sphere of radius D/2, polar angle kappa from the tip up
 * to the depth of cut plus the tilt. */
static void edge_point(const or_tool *t, const or_cut *c, int p, double pc[4])
{
    const int N = t->n_edge;
    if (t->kind == 0) {
        const double R = t->R_edge;
        double dL_ap = R;
        if (c->a_p < R) dL_ap = sqrt(R * R - (R - c->a_p) * (R - c->a_p));
        const double dL_fz = c->f_z / (2.0 * cos(t->rake_f));
        double dL = dL_ap > dL_fz ? dL_ap : dL_fz;
        if (dL > R) dL = R;
        double l = 0.0;
        if (N > 1) l = -dL + ((2.0 * dL) / (double)(N - 1)) * (double)p;
        pc[0] = l;
        pc[1] = 0.0;
        pc[2] = R - sqrt(R * R - l * l);
    } else {
        const double Rb = t->D / 2.0;
        double u = 1.0 - c->a_p / Rb;
        if (u < 0.0) u = 0.0;
        double kmax = (fabs(t->tilt_lead) + fabs(t->tilt_side)) + acos(u);
        if (kmax > M_PI / 2.0) kmax = M_PI / 2.0;
        double k = 0.0;
        if (N > 1) k = (kmax * (double)p) / (double)(N - 1);
        pc[0] = Rb * sin(k);
        pc[1] = 0.0;
        pc[2] = Rb * (1.0 - cos(k));
    }
    pc[3] = 1.0;
}

/* Eq. (2) for tooth K: rake rotation plus the translation to the cutting diameter with the
 * per-insert runout.  The ball profile is already expressed about the tool axis, so its
 * translation carries only the runout. */
static void m_edge_to_tool(const or_tool *t, int K, m4 M)
{
    const double cf = cos(t->rake_f), sf = sin(t->rake_f);
    const double cp = cos(t->rake_p), sp = sin(t->rake_p);
    const double off = t->kind == 0 ? t->D / 2.0 : 0.0;
    m_identity(M);
    M[0][0] = cf;  M[0][1] = sf * cp; M[0][2] = sf * sp; M[0][3] = off + t->eps_r[K];
    M[1][0] = -sf; M[1][1] = cf * cp; M[1][2] = cf * sp; M[1][3] = 0.0;
    M[2][0] = 0.0; M[2][1] = -sp;     M[2][2] = cp;      M[2][3] = t->eps_a[K];
}

/* Rotation about the tool axis with the matrix layout of Eq. (3):
 * [[cos a, sin a], [-sin a, cos a]], i.e. a turn by -a. */
static void m_rot_z(double a, m4 M)
{
    m_identity(M);
    const double ca = cos(a), sa = sin(a);
    M[0][0] = ca;  M[0][1] = sa;
    M[1][0] = -sa; M[1][1] = ca;
}

int or_edge_points(const or_tool *t, const or_cut *c, double *pC, double *pT)
{
    if (check_tool(t) || check_cut(c)) return -1;
    const int N = t->n_edge;
    for (int p = 0; p < N; ++p) {
        double pc[4];
        edge_point(t, c, p, pc);
        if (pC) { pC[3 * p] = pc[0]; pC[3 * p + 1] = pc[1]; pC[3 * p + 2] = pc[2]; }
    }
    if (!pT) return 0;
    const double tanb = tan(t->helix);
    const double Rref = t->D / 2.0;
    for (int K = 0; K < t->n_teeth; ++K) {
        m4 C;
        m_edge_to_tool(t, K, C);
        /* The eccentric offset is a vector (e cos lambda, e sin lambda) fixed in the cutter
         * body.  Tooth K's frame trails the body by theta_K, so in that frame the vector
         * has phase lambda + theta_K. */
        m4 E;
        m_identity(E);
        const double ph = t->ecc_phase + tooth_angle(t, K);
        E[0][3] = t->ecc * cos(ph);
        E[1][3] = t->ecc * sin(ph);
        for (int p = 0; p < N; ++p) {
            double pc[4], a[4], b[4], r[4];
            edge_point(t, c, p, pc);
            mv(C, pc, a);
            m4 H;
            m_rot_z((pc[2] * tanb) / Rref, H);   /* helix lag: trailing turn by psi */
            mv(H, a, b);
            mv(E, b, r);
            double *o = pT + 3 * ((long long)K * N + p);
            o[0] = r[0]; o[1] = r[1]; o[2] = r[2];
        }
    }
    return 0;
}

/* ---- plan: travel extent, passes and steps ----------------------------------------------- */

int or_plan(const or_tool *t, const or_cut *c, const or_grid *g, or_plan_out *out)
{
    if (check_tool(t) || check_cut(c) || check_grid(g) || !out) return -1;
    const int N = t->n_edge, Z = t->n_teeth;
    double *pT = (double *)malloc(sizeof(double) * 3 * (size_t)N * (size_t)Z);
    if (!pT) return -2;
    or_edge_points(t, c, NULL, pT);
    const double sl = fabs(sin(t->tilt_lead)), ss = fabs(sin(t->tilt_side));
    double reach = 0.0;
    for (long long k = 0; k < (long long)N * Z; ++k) {
        const double x = pT[3 * k], y = pT[3 * k + 1], z = pT[3 * k + 2];
        const double r = sqrt(x * x + y * y) + fabs(z) * (sl + ss);
        if (r > reach) reach = r;
    }
    free(pT);

    const double x_lo = g->x0 - 0.5 * g->dd, y_lo = g->y0 - 0.5 * g->dd;
    const double x_hi = x_lo + (double)g->nx * g->dd, y_hi = y_lo + (double)g->ny * g->dd;
    const double fpr = (double)Z * c->f_z;

    out->r_reach = reach;
    out->x_start = isnan(c->x_start) ? x_lo - reach : c->x_start;
    const double x_end = isnan(c->x_end) ? x_hi + reach : c->x_end;
    if (c->n_steps > 0) {
        out->n_steps = c->n_steps;
    } else if (c->time_mode == 1) {
        /* time over the travel at the feed speed, in whole time steps */
        const double v_f = feed_speed(t, c);
        double steps = v_f > 0.0 ? ceil(((x_end - out->x_start) / v_f) / c->dt) : 1.0;
        if (steps < 1.0) steps = 1.0;
        out->n_steps = (long long)steps;
    } else if (fpr > 0.0) {
        double revs = ceil((x_end - out->x_start) / fpr);
        if (revs < 1.0) revs = 1.0;
        out->n_steps = (long long)revs * c->S;
    } else {
        out->n_steps = c->S;
    }
    if (c->n_passes > 0) {
        out->n_passes = c->n_passes;
    } else if (c->a_e > 0.0) {
        out->n_passes = (long long)ceil(((y_hi + reach) - (y_lo - reach)) / c->a_e) + 1;
    } else {
        out->n_passes = 1;
    }
    if (!isnan(c->y_first)) out->y_first = c->y_first;
    else if (c->a_e > 0.0) out->y_first = y_lo - reach;
    else out->y_first = g->y0 + 0.5 * (double)(g->ny - 1) * g->dd;
    out->n_evals = out->n_passes * out->n_steps * Z * N;
    return 0;
}

/* ---- kinematics -------------------------------------------------------------------------- */

typedef struct chain {
    or_plan_out plan;
    double *pT;          /* [Z][N][3] */
    m4 Ry, Rx;           /* tilt */
    double fpr;
    double omega, v_f;   /* fixed-time-step mode */
} chain;

static int chain_init(const or_tool *t, const or_cut *c, const or_grid *g, chain *ch)
{
    int rc = or_plan(t, c, g, &ch->plan);
    if (rc) return rc;
    ch->pT = (double *)malloc(sizeof(double) * 3 * (size_t)t->n_edge * (size_t)t->n_teeth);
    if (!ch->pT) return -2;
    or_edge_points(t, c, NULL, ch->pT);
    const double cl = cos(t->tilt_lead), sl = sin(t->tilt_lead);
    const double cs = cos(t->tilt_side), ss = sin(t->tilt_side);
    m_identity(ch->Ry);
    ch->Ry[0][0] = cl;  ch->Ry[0][2] = sl;
    ch->Ry[2][0] = -sl; ch->Ry[2][2] = cl;
    m_identity(ch->Rx);
    ch->Rx[1][1] = cs; ch->Rx[1][2] = -ss;
    ch->Rx[2][1] = ss; ch->Rx[2][2] = cs;
    ch->fpr = (double)t->n_teeth * c->f_z;
    ch->omega = c->time_mode == 1 ? omega_of(t, c) : 0.0;
    ch->v_f = c->time_mode == 1 ? feed_speed(t, c) : 0.0;
    return 0;
}

/* Eq. (4) read with the feed along X: tool centre at step s of pass q (v_f t at t = s dt in
 * the fixed-time-step mode). */
static void m_spindle_to_work(const or_cut *c, const chain *ch, long long q, long long s, m4 W)
{
    m_identity(W);
    if (c->time_mode == 1)
        W[0][3] = ch->plan.x_start + ch->v_f * ((double)s * c->dt);
    else
        W[0][3] = ch->plan.x_start + ((double)s * ch->fpr) / (double)c->S;
    W[1][3] = ch->plan.y_first + (double)q * c->a_e;
}

/* Eq. (3): alpha = phi + 2 pi (K-1)/z_n - omega t, with omega t = 2 pi (s mod S) / S, or
 * omega (s dt) in the fixed-time-step mode. */
static void m_tool_to_spindle(const or_tool *t, const or_cut *c, const chain *ch, long long s,
                              int K, m4 T)
{
    double alpha;
    if (c->time_mode == 1)
        alpha = (c->phi0 + tooth_angle(t, K)) - ch->omega * ((double)s * c->dt);
    else
        alpha = (c->phi0 + tooth_angle(t, K)) - ((2.0 * M_PI) * (double)(s % c->S)) / (double)c->S;
    m_rot_z(alpha, T);
}

static void transform(const chain *ch, const m4 T, const m4 W, const double *pt, double w[4])
{
    double v[4] = {pt[0], pt[1], pt[2], 1.0}, a[4], b[4], d[4];
    mv(T, v, a);
    mv(ch->Ry, a, b);
    mv(ch->Rx, b, d);
    mv(W, d, w);
}

int or_point(const or_tool *t, const or_cut *c, const or_grid *g,
             long long q, long long s, int K, int p, double out[3])
{
    chain ch;
    int rc = chain_init(t, c, g, &ch);
    if (rc) return rc;
    if (K < 0 || K >= t->n_teeth || p < 0 || p >= t->n_edge) { free(ch.pT); return -1; }
    m4 T, W;
    m_tool_to_spindle(t, c, &ch, s, K, T);
    m_spindle_to_work(c, &ch, q, s, W);
    double w[4];
    transform(&ch, T, W, ch.pT + 3 * ((long long)K * t->n_edge + p), w);
    out[0] = w[0]; out[1] = w[1]; out[2] = w[2];
    free(ch.pT);
    return 0;
}

/* The trajectory module of Sec. 3.2: at every time step, the lowest point (least z) of each
 * tooth's discretised edge in the workpiece frame; the first such point on a tie. */
int or_trajectory(const or_tool *t, const or_cut *c, const or_grid *g, double *xyz, int *idx)
{
    if (!xyz) return -1;
    chain ch;
    int rc = chain_init(t, c, g, &ch);
    if (rc) return rc;
    const int Zt = t->n_teeth, N = t->n_edge;
    for (long long q = 0; q < ch.plan.n_passes; ++q) {
        for (long long s = 0; s < ch.plan.n_steps; ++s) {
            m4 W;
            m_spindle_to_work(c, &ch, q, s, W);
            for (int K = 0; K < Zt; ++K) {
                m4 T;
                m_tool_to_spindle(t, c, &ch, s, K, T);
                double best[4] = {0.0, 0.0, INFINITY, 1.0};
                int bp = -1;
                for (int p = 0; p < N; ++p) {
                    double w[4];
                    transform(&ch, T, W, ch.pT + 3 * ((long long)K * N + p), w);
                    if (w[2] < best[2]) {
                        best[0] = w[0]; best[1] = w[1]; best[2] = w[2];
                        bp = p;
                    }
                }
                const long long o = (q * ch.plan.n_steps + s) * Zt + K;
                xyz[3 * o] = best[0];
                xyz[3 * o + 1] = best[1];
                xyz[3 * o + 2] = best[2];
                if (idx) idx[o] = bp;
            }
        }
    }
    free(ch.pT);
    return 0;
}

/* Eq. (7) with half-open sampling boundaries [x_i - dd/2, x_i + dd/2): the node index is the
 * floor of the offset from the lower boundary in units of dd.  Returns 0 when the point lies
 * outside the grid (such points are dropped, not clamped). */
static int bin(const or_grid *g, double x_lo, double y_lo, double inv, const double w[4],
               long long *i, long long *j)
{
    const double fi = floor((w[0] - x_lo) * inv);
    const double fj = floor((w[1] - y_lo) * inv);
    if (!(fi >= 0.0 && fi < (double)g->nx && fj >= 0.0 && fj < (double)g->ny)) return 0;
    *i = (long long)fi;
    *j = (long long)fj;
    return 1;
}

int or_simulate_window(const or_tool *t, const or_cut *c, const or_grid *g,
                       long long i0, long long i1, long long j0, long long j1,
                       double *Zw, long long *win, or_counts *cnt)
{
    if (i0 < 0 || j0 < 0 || i1 > g->nx || j1 > g->ny || i0 > i1 || j0 > j1 || !Zw) return -1;
    chain ch;
    int rc = chain_init(t, c, g, &ch);
    if (rc) return rc;
    const long long wx = i1 - i0, wy = j1 - j0;
    for (long long k = 0; k < wx * wy; ++k) Zw[k] = INFINITY;
    if (win) for (long long k = 0; k < wx * wy; ++k) win[k] = -1;

    const double x_lo = g->x0 - 0.5 * g->dd, y_lo = g->y0 - 0.5 * g->dd, inv = 1.0 / g->dd;
    const int Zt = t->n_teeth, N = t->n_edge;
    long long n_binned = 0;
    for (long long q = 0; q < ch.plan.n_passes; ++q) {
        for (long long s = 0; s < ch.plan.n_steps; ++s) {
            m4 W;
            m_spindle_to_work(c, &ch, q, s, W);
            for (int K = 0; K < Zt; ++K) {
                m4 T;
                m_tool_to_spindle(t, c, &ch, s, K, T);
                for (int p = 0; p < N; ++p) {
                    double w[4];
                    transform(&ch, T, W, ch.pT + 3 * ((long long)K * N + p), w);
                    long long i, j;
                    if (!bin(g, x_lo, y_lo, inv, w, &i, &j)) continue;
                    ++n_binned;
                    if (i < i0 || i >= i1 || j < j0 || j >= j1) continue;
                    const long long k = (j - j0) * wx + (i - i0);
                    if (w[2] < Zw[k]) {
                        Zw[k] = w[2];
                        if (win) win[k] = ((q * ch.plan.n_steps + s) * Zt + K) * N + p;
                    }
                }
            }
        }
    }
    if (cnt) { cnt->n_evals = ch.plan.n_evals; cnt->n_binned = n_binned; }
    free(ch.pT);
    return 0;
}

/* Interval of each cell's minimum when every evaluation's workpiece position (x, y) may move by
 * up to `delta` along each axis: the cell-assignment rule of Eq. (7) applied to every position
 * in the square [x - delta, x + delta] x [y - delta, y + delta].  lo: least height of an
 * evaluation that can reach the cell; hi: least height of one that reaches it wherever it
 * moves (+inf if none); top: greatest height of one that can reach it (-inf if none).  Any
 * per-cell minimum over moved positions is +inf or lies in [lo, min(hi, top)], and is finite
 * whenever hi is.  With delta = 0, lo and hi equal the Z-map. */
int or_cell_bounds_window(const or_tool *t, const or_cut *c, const or_grid *g, double delta,
                          long long i0, long long i1, long long j0, long long j1,
                          double *lo, double *hi, double *top)
{
    if (!lo || !hi || !top || !(delta >= 0.0)) return -1;
    if (i0 < 0 || j0 < 0 || i1 > g->nx || j1 > g->ny || i0 >= i1 || j0 >= j1) return -1;
    chain ch;
    int rc = chain_init(t, c, g, &ch);
    if (rc) return rc;
    const long long wx = i1 - i0, cells = wx * (j1 - j0);
    for (long long k = 0; k < cells; ++k) {
        lo[k] = INFINITY;
        hi[k] = INFINITY;
        top[k] = -INFINITY;
    }
    const double x_lo = g->x0 - 0.5 * g->dd, y_lo = g->y0 - 0.5 * g->dd, inv = 1.0 / g->dd;
    const double dr = delta * inv;
    const int Zt = t->n_teeth, N = t->n_edge;
    for (long long q = 0; q < ch.plan.n_passes; ++q) {
        for (long long s = 0; s < ch.plan.n_steps; ++s) {
            m4 W;
            m_spindle_to_work(c, &ch, q, s, W);
            for (int K = 0; K < Zt; ++K) {
                m4 T;
                m_tool_to_spindle(t, c, &ch, s, K, T);
                for (int p = 0; p < N; ++p) {
                    double w[4];
                    transform(&ch, T, W, ch.pT + 3 * ((long long)K * N + p), w);
                    const double fx = (w[0] - x_lo) * inv, fy = (w[1] - y_lo) * inv;
                    const double ia = floor(fx - dr), ib = floor(fx + dr);
                    const double ja = floor(fy - dr), jb = floor(fy + dr);
                    const int sure = ia == ib && ja == jb;
                    for (double fj = ja; fj <= jb; fj += 1.0) {
                        for (double fi = ia; fi <= ib; fi += 1.0) {
                            if (fi < (double)i0 || fj < (double)j0 || fi >= (double)i1 || fj >= (double)j1)
                                continue;
                            const long long k = ((long long)fj - j0) * wx + ((long long)fi - i0);
                            if (w[2] < lo[k]) lo[k] = w[2];
                            if (w[2] > top[k]) top[k] = w[2];
                            if (sure && w[2] < hi[k]) hi[k] = w[2];
                        }
                    }
                }
            }
        }
    }
    free(ch.pT);
    return 0;
}

int or_cell_bounds(const or_tool *t, const or_cut *c, const or_grid *g, double delta,
                   double *lo, double *hi, double *top)
{
    return or_cell_bounds_window(t, c, g, delta, 0, g->nx, 0, g->ny, lo, hi, top);
}

/* ---- roughness --------------------------------------------------------------------------- */

/* Arithmetic-mean height of the hit cells along one line, and the mean absolute deviation
 * about it (profile Ra). */
static void profile_ra(const double *Z, long long start, long long stride, long long n,
                       double *ra, long long *cnt)
{
    long long m = 0;
    double sum = 0.0;
    for (long long k = 0; k < n; ++k) {
        const double z = Z[start + k * stride];
        if (z < INFINITY) { sum += z; ++m; }
    }
    *cnt = m;
    if (m == 0) { *ra = NAN; return; }
    const double mu = sum / (double)m;
    double a = 0.0;
    for (long long k = 0; k < n; ++k) {
        const double z = Z[start + k * stride];
        if (z < INFINITY) a += fabs(z - mu);
    }
    *ra = a / (double)m;
}

/* Areal parameters over the hit cells with the arithmetic mean as reference plane:
 * Sa = mean|d|, Sq = sqrt(mean d^2), Sp = max - mean, Sv = mean - min, Sz = Sp + Sv,
 * Ssk = mean d^3 / Sq^3, Sku = mean d^4 / Sq^4, d = z - mean. */
int or_roughness(const double *Z, long long nx, long long ny, or_rough *r)
{
    if (!Z || !r || nx < 1 || ny < 1) return -1;
    const long long n = nx * ny;
    long long m = 0;
    double sum = 0.0, mn = INFINITY, mx = -INFINITY;
    for (long long k = 0; k < n; ++k) {
        const double z = Z[k];
        if (!(z < INFINITY)) continue;
        ++m;
        sum += z;
        if (z < mn) mn = z;
        if (z > mx) mx = z;
    }
    r->n_hit = m;
    if (m == 0) {
        r->Sa = r->Sq = r->Sp = r->Sv = r->Sz = r->Ssk = r->Sku = r->mean = NAN;
    } else {
        const double mu = sum / (double)m;
        double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
        for (long long k = 0; k < n; ++k) {
            const double z = Z[k];
            if (!(z < INFINITY)) continue;
            const double d = z - mu;
            s1 += fabs(d);
            s2 += d * d;
            s3 += d * d * d;
            s4 += d * d * d * d;
        }
        r->mean = mu;
        r->Sa = s1 / (double)m;
        r->Sq = sqrt(s2 / (double)m);
        r->Sp = mx - mu;
        r->Sv = mu - mn;
        r->Sz = r->Sp + r->Sv;
        if (r->Sq > 0.0) {
            r->Ssk = (s3 / (double)m) / (r->Sq * r->Sq * r->Sq);
            r->Sku = (s4 / (double)m) / (r->Sq * r->Sq * r->Sq * r->Sq);
        } else {
            r->Ssk = r->Sku = NAN;
        }
    }
    profile_ra(Z, (ny / 2) * nx, 1, nx, &r->Ra_feed, &r->n_feed);
    profile_ra(Z, nx / 2, nx, ny, &r->Ra_pick, &r->n_pick);
    return 0;
}

/* ---- the paper's fixed-time-step mode ---------------------------------------------------- */

long long or_paper_trajectory_points(double v_c, double f_z, int z_n, double D,
                                     double L, double dt)
{
    if (!(v_c > 0.0) || !(f_z > 0.0) || z_n < 1 || !(D > 0.0) || !(L > 0.0) || !(dt > 0.0))
        return -1;
    const double n_rpm = (1000.0 * v_c) / (M_PI * D);   /* spindle speed from cutting speed */
    const double v_f = (f_z * (double)z_n * n_rpm) / 60.0; /* feed speed, mm/s */
    const double T = L / v_f;                             /* machining time over the length */
    const long long steps = (long long)ceil(T / dt);
    return (long long)z_n * steps;                        /* one trajectory point per tooth per step */
}

/* ---- surface-texture operators (measurement practice of Sec. 4.1.1) ----------------------- */

/* Least-squares plane: the normal equations (A^T A) c = A^T z of the design rows (1, x, y),
 * solved by Gaussian elimination with partial pivoting. */
int or_level(const double *Z, const or_grid *g, double *out, double *plane)
{
    if (!Z || !g || !out || g->nx < 1 || g->ny < 1 || !(g->dd > 0.0)) return -1;
    double M[3][4] = {{0.0}};
    for (long long j = 0; j < g->ny; ++j) {
        for (long long i = 0; i < g->nx; ++i) {
            const double z = Z[j * g->nx + i];
            if (!(z < INFINITY)) continue;
            const double r[3] = {1.0, g->x0 + (double)i * g->dd, g->y0 + (double)j * g->dd};
            for (int a = 0; a < 3; ++a) {
                for (int b = 0; b < 3; ++b) M[a][b] += r[a] * r[b];
                M[a][3] += r[a] * z;
            }
        }
    }
    if (M[0][0] < 3.0) return -2;
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (!(fabs(M[piv][col]) > 1e-12 * M[0][0])) return -2;
        if (piv != col)
            for (int k = 0; k < 4; ++k) {
                const double tmp = M[col][k];
                M[col][k] = M[piv][k];
                M[piv][k] = tmp;
            }
        for (int r = col + 1; r < 3; ++r) {
            const double f = M[r][col] / M[col][col];
            for (int k = col; k < 4; ++k) M[r][k] -= f * M[col][k];
        }
    }
    double c[3];
    for (int r = 2; r >= 0; --r) {
        double v = M[r][3];
        for (int k = r + 1; k < 3; ++k) v -= M[r][k] * c[k];
        c[r] = v / M[r][r];
    }
    for (long long j = 0; j < g->ny; ++j) {
        for (long long i = 0; i < g->nx; ++i) {
            const long long k = j * g->nx + i;
            const double z = Z[k];
            out[k] = z < INFINITY
                ? z - (c[0] + c[1] * (g->x0 + (double)i * g->dd) + c[2] * (g->y0 + (double)j * g->dd))
                : INFINITY;
        }
    }
    if (plane) {
        plane[0] = c[0];
        plane[1] = c[1];
        plane[2] = c[2];
    }
    return 0;
}

static long long gauss_radius(const or_grid *g, double lambda, double trunc)
{
    return (long long)floor(trunc * lambda / g->dd + 1e-9);
}

/* weights w[a] = exp(-pi (a dd / (alpha lambda))^2), a = 0..R */
static double *gauss_weights(const or_grid *g, double lambda, long long R)
{
    double *w = (double *)malloc(sizeof(double) * (size_t)(R + 1));
    if (!w) return NULL;
    const double alpha = sqrt(log(2.0) / M_PI);
    for (long long a = 0; a <= R; ++a) {
        const double u = ((double)a * g->dd) / (alpha * lambda);
        w[a] = exp(-M_PI * (u * u));
    }
    return w;
}

static double gauss_cell(const double *Z, const or_grid *g, const double *w, long long R,
                         int mode, long long i, long long j)
{
    const double z = Z[j * g->nx + i];
    if (!(z < INFINITY)) return INFINITY;
    double num = 0.0, den = 0.0;
    for (long long b = -R; b <= R; ++b) {
        const long long jj = j + b;
        if (jj < 0 || jj >= g->ny) continue;
        for (long long a = -R; a <= R; ++a) {
            const long long ii = i + a;
            if (ii < 0 || ii >= g->nx) continue;
            const double v = Z[jj * g->nx + ii];
            if (!(v < INFINITY)) continue;
            const double wt = w[a < 0 ? -a : a] * w[b < 0 ? -b : b];
            num += wt * v;
            den += wt;
        }
    }
    const double mean = num / den;
    return mode == 0 ? mean : z - mean;
}

static int gauss_check(const double *Z, const or_grid *g, double lambda, double trunc, int mode)
{
    if (!Z || !g || g->nx < 1 || g->ny < 1 || !(g->dd > 0.0) || !(lambda > 0.0) ||
        !(trunc > 0.0) || !(trunc <= 4.0) || (mode != 0 && mode != 1))
        return -1;
    return 0;
}

int or_gauss_filter(const double *Z, const or_grid *g, double lambda, double trunc, int mode,
                    double *out)
{
    if (gauss_check(Z, g, lambda, trunc, mode) || !out || out == Z) return -1;
    const long long R = gauss_radius(g, lambda, trunc);
    double *w = gauss_weights(g, lambda, R);
    if (!w) return -3;
    for (long long j = 0; j < g->ny; ++j)
        for (long long i = 0; i < g->nx; ++i)
            out[j * g->nx + i] = gauss_cell(Z, g, w, R, mode, i, j);
    free(w);
    return 0;
}

int or_gauss_filter_cells(const double *Z, const or_grid *g, double lambda, double trunc,
                          int mode, const long long *cells, long long n, double *out)
{
    if (gauss_check(Z, g, lambda, trunc, mode) || !cells || !out || n < 0) return -1;
    for (long long k = 0; k < n; ++k)
        if (cells[k] < 0 || cells[k] >= g->nx * g->ny) return -1;
    const long long R = gauss_radius(g, lambda, trunc);
    double *w = gauss_weights(g, lambda, R);
    if (!w) return -3;
    for (long long k = 0; k < n; ++k)
        out[k] = gauss_cell(Z, g, w, R, mode, cells[k] % g->nx, cells[k] / g->nx);
    free(w);
    return 0;
}
