/* The C ABI used from C: the header compiles as C11, the library links, and the host-only
 * calls (version, planning, edge points, refinement, error strings) behave as declared. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "fsm.h"

#define CHECK(c)                                              \
    do {                                                      \
        if (!(c)) {                                           \
            printf("FAIL line %d: %s\n", __LINE__, #c);       \
            return 1;                                         \
        }                                                     \
    } while (0)

int main(void)
{
    CHECK(fsm_version() >= 1);
    fsm_tool t;
    memset(&t, 0, sizeof t);
    t.kind = FSM_TOOL_ROUND;
    t.n_teeth = 2;
    t.n_edge = 12;
    t.uniform_pitch = 1;
    t.D = 2.0;
    t.R_edge = 1.0;
    fsm_cut c;
    memset(&c, 0, sizeof c);
    c.f_z = 0.05;
    c.a_p = 0.2;
    c.steps_per_rev = 90;
    c.n_passes = 1;
    c.x_start = NAN;
    c.y_first = 0.0;
    c.x_end = NAN;
    fsm_grid g = {-0.295, -0.295, 0.01, 60, 60};
    fsm_plan_info info;
    CHECK(fsm_plan(&t, &c, &g, FSM_F64, &info) == FSM_OK);
    CHECK(info.n_passes == 1 && info.n_steps > 0);
    CHECK(info.n_evals == (int64_t)t.n_teeth * t.n_edge * info.n_steps * info.n_passes);
    double pts[2 * 12 * 3];
    CHECK(fsm_edge_points(&t, &c, pts) == FSM_OK);
    for (int k = 0; k < 2 * 12 * 3; ++k) CHECK(isfinite(pts[k]));
    fsm_tool t2;
    fsm_cut c2;
    CHECK(fsm_refine(&t, &c, &g, 0.005, &t2, &c2) == FSM_OK);
    CHECK(t2.n_edge >= t.n_edge && c2.steps_per_rev >= c.steps_per_rev && c2.n_steps == 0);
    /* bad arguments come back as status codes */
    CHECK(fsm_plan(NULL, &c, &g, FSM_F64, &info) == FSM_EINVAL);
    CHECK(fsm_refine(&t, &c, &g, -1.0, &t2, &c2) == FSM_EINVAL);
    t.n_teeth = 0;
    CHECK(fsm_plan(&t, &c, &g, FSM_F64, &info) == FSM_EINVAL);
    CHECK(strlen(fsm_strerror(FSM_EINVAL)) > 0 && strlen(fsm_strerror(FSM_EAGAIN)) > 0);
    printf("OK\n");
    return 0;
}
