"""Mutation tests of the oracle's pins.  Each case plants one plausible mistake in a copy of
the oracle's C source (a flipped sign, a dropped term, a wrong index or boundary), builds it
with the oracle's own flags, runs the pin battery (tests/test_oracle_pins.py, the oracle
checks of tests/test_f32_bounds.py and the texture pins of tests/test_texture_pins.py) on it
and requires at least one pin to fail.  Every planted mistake stays memory-safe.  CPU only."""
import inspect
import os
import subprocess

import pytest

import oracle

import test_f32_bounds as bounds_pins
import test_oracle_pins as pins
import test_texture_pins as texture_pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "fsm_oracle.c")

# (name, [(text, replacement), ...]) -- each text occurs exactly once in the source
MUTANTS = [
    ("rotation sense of Eq. (3)",
     [("M[0][0] = ca;  M[0][1] = sa;\n    M[1][0] = -sa; M[1][1] = ca;",
       "M[0][0] = ca;  M[0][1] = -sa;\n    M[1][0] = sa; M[1][1] = ca;")]),
    ("per-insert radial offset inward",
     [("M[0][3] = off + t->eps_r[K];", "M[0][3] = off - t->eps_r[K];")]),
    ("per-insert axial offset upward",
     [("M[2][3] = t->eps_a[K];", "M[2][3] = -t->eps_a[K];")]),
    ("variable pitch ignored",
     [("if (t->uniform_pitch) return", "if (1) return")]),
    ("peak height from zero, not from the mean",
     [("r->Sp = mx - mu;", "r->Sp = mx;")]),
    ("arithmetic mean deviation without the absolute value",
     [("s1 += fabs(d);", "s1 += d;")]),
    ("feed-direction profile taken along a column",
     [("profile_ra(Z, (ny / 2) * nx, 1, nx, &r->Ra_feed, &r->n_feed);",
       "profile_ra(Z, nx / 2, nx, ny, &r->Ra_feed, &r->n_feed);")]),
    ("eccentric runout phased by the uniform pitch for variable-pitch teeth",
     [("const double ph = t->ecc_phase + tooth_angle(t, K);",
       "const double ph = t->ecc_phase + ((2.0 * M_PI) * (double)K) / (double)t->n_teeth;")]),
    ("per-insert offsets taken by position, not by insert",
     [("M[0][3] = off + t->eps_r[K];", "M[0][3] = off + (double)K * t->eps_r[1];")]),
    ("tooth phase sign",
     [("return ((2.0 * M_PI) * (double)K) / (double)t->n_teeth;",
       "return -((2.0 * M_PI) * (double)K) / (double)t->n_teeth;")]),
    ("time runs backwards",
     [("- ((2.0 * M_PI) * (double)(s % c->S)) / (double)c->S;",
       "+ ((2.0 * M_PI) * (double)(s % c->S)) / (double)c->S;")]),
    ("feed per revolution without z_n",
     [("ch->fpr = (double)t->n_teeth * c->f_z;", "ch->fpr = c->f_z;")]),
    ("half the stepover",
     [("W[1][3] = ch->plan.y_first + (double)q * c->a_e;",
       "W[1][3] = ch->plan.y_first + (double)q * c->a_e * 0.5;")]),
    ("rounded instead of floored cell index",
     [("const double fi = floor((w[0] - x_lo) * inv);",
       "const double fi = round((w[0] - x_lo) * inv);")]),
    ("first grid column dropped",
     [("if (!(fi >= 0.0 && fi < (double)g->nx", "if (!(fi >= 1.0 && fi < (double)g->nx")]),
    ("helix lag leads instead of trails",
     [("m_rot_z((pc[2] * tanb) / Rref, H);", "m_rot_z(-(pc[2] * tanb) / Rref, H);")]),
    ("eccentric runout in each tooth's own frame",
     [("const double ph = t->ecc_phase + tooth_angle(t, K);", "const double ph = t->ecc_phase;")]),
    ("lead tilt sign",
     [("ch->Ry[0][0] = cl;  ch->Ry[0][2] = sl;\n    ch->Ry[2][0] = -sl;",
       "ch->Ry[0][0] = cl;  ch->Ry[0][2] = -sl;\n    ch->Ry[2][0] = sl;")]),
    ("side tilt sign",
     [("ch->Rx[1][1] = cs; ch->Rx[1][2] = -ss;\n    ch->Rx[2][1] = ss;",
       "ch->Rx[1][1] = cs; ch->Rx[1][2] = ss;\n    ch->Rx[2][1] = -ss;")]),
    ("rake turn sign",
     [("M[0][0] = cf;  M[0][1] = sf * cp;", "M[0][0] = cf;  M[0][1] = -sf * cp;"),
      ("M[1][0] = -sf; M[1][1] = cf * cp;", "M[1][0] = sf; M[1][1] = cf * cp;")]),
    ("feed-limited chord without the rake",
     [("c->f_z / (2.0 * cos(t->rake_f))", "c->f_z / 2.0")]),
    ("ball meridian off the sphere",
     [("pc[2] = Rb * (1.0 - cos(k));", "pc[2] = Rb * (1.0 - cos(k)) * 0.99;")]),
    ("reach without the tilt",
     [("const double r = sqrt(x * x + y * y) + fabs(z) * (sl + ss);",
       "const double r = sqrt(x * x + y * y);")]),
    ("maximum instead of minimum",
     [("if (w[2] < Zw[k]) {", "if (w[2] > Zw[k] || Zw[k] == INFINITY) {")]),
    ("sample instead of population variance",
     [("r->Sq = sqrt(s2 / (double)m);", "r->Sq = sqrt(s2 / (double)(m > 1 ? m - 1 : 1));")]),
    ("kurtosis normalised by Sq cubed",
     [("r->Sku = (s4 / (double)m) / (r->Sq * r->Sq * r->Sq * r->Sq);",
       "r->Sku = (s4 / (double)m) / (r->Sq * r->Sq * r->Sq);")]),
    ("skewness sign",
     [("r->Ssk = (s3 / (double)m) / (r->Sq * r->Sq * r->Sq);",
       "r->Ssk = -(s3 / (double)m) / (r->Sq * r->Sq * r->Sq);")]),
    ("fixed-step spindle speed without 2 pi",
     [("return ((2.0 * M_PI) * spindle_rpm(t, c)) / 60.0;", "return spindle_rpm(t, c) / 60.0;")]),
    ("fixed-step feed speed without z_n",
     [("return (c->f_z * (double)t->n_teeth * spindle_rpm(t, c)) / 60.0;",
       "return (c->f_z * spindle_rpm(t, c)) / 60.0;")]),
    ("trajectory counts per step, not per tooth and step",
     [("return (long long)z_n * steps;", "return steps;")]),
    ("trajectory ties won by the last point",
     [("if (w[2] < best[2]) {", "if (w[2] <= best[2]) {")]),
    ("trajectory keeps the highest point",
     [("                    if (w[2] < best[2]) {", "                    if (!(w[2] <= best[2]) || bp < 0) {")]),
    ("interval: every candidate counted as certain",
     [("const int sure = ia == ib && ja == jb;", "const int sure = 1;")]),
    ("interval: certain points not counted as reachable",
     [("if (w[2] < lo[k]) lo[k] = w[2];", "if (!sure && w[2] < lo[k]) lo[k] = w[2];")]),
    ("Gaussian width without the square root",
     [("const double alpha = sqrt(log(2.0) / M_PI);", "const double alpha = log(2.0) / M_PI;")]),
    ("Gaussian y weight indexed by x",
     [("w[a < 0 ? -a : a] * w[b < 0 ? -b : b]", "w[a < 0 ? -a : a] * w[a < 0 ? -a : a]")]),
    ("empty cells weighted in the filter",
     [("            if (!(v < INFINITY)) continue;\n", "")]),
    ("Gaussian window one cell short on the right",
     [("for (long long a = -R; a <= R; ++a) {", "for (long long a = -R; a < R; ++a) {")]),
    ("Gaussian border renormalised as if columns beyond the right edge were hit",
     [("if (ii < 0 || ii >= g->nx) continue;",
       "if (ii < 0) continue;\n            if (ii >= g->nx) { den += w[a < 0 ? -a : a] * w[b < 0 ? -b : b]; continue; }")]),
    ("high-pass sign",
     [("return mode == 0 ? mean : z - mean;", "return mode == 0 ? mean : mean - z;")]),
    ("plane y term evaluated at the column",
     [("c[2] * (g->y0 + (double)j * g->dd))", "c[2] * (g->y0 + (double)i * g->dd))")]),
    ("normal equations without the cross term",
     [("for (int b = 0; b < 3; ++b) M[a][b] += r[a] * r[b];",
       "for (int b = 0; b < 3; ++b) M[a][b] += a == b ? r[a] * r[b] : 0.0;")]),
]


def battery():
    """Every pin as a zero-argument call, cheapest first (parametrised pins expanded)."""
    calls = []
    for mod in (pins, bounds_pins, texture_pins):
        for name, f in inspect.getmembers(mod, inspect.isfunction):
            if not name.startswith("test_") or f.__module__ != mod.__name__:
                continue
            marks = [m for m in getattr(f, "pytestmark", []) if m.name == "parametrize"]
            if not marks:
                calls.append((name, f, {}))
                continue
            argname, values = marks[0].args[0], marks[0].args[1]
            for v in values:
                calls.append((f"{name}[{v}]", f, {argname: v}))
    slow = {"test_adding_pass_never_raises"}
    return sorted(calls, key=lambda c: c[0] in slow)


def build_mutant(tmp_path, subs):
    text = open(SRC).read()
    for old, new in subs:
        assert text.count(old) == 1, old
        text = text.replace(old, new)
    src = tmp_path / "mutant.c"
    src.write_text(text)
    lib = tmp_path / "libmutant.so"
    hdr_dir = os.path.dirname(SRC)
    subprocess.run(["gcc", *oracle.oracle.CFLAGS, "-I", hdr_dir, "-o", str(lib), str(src), "-lm"],
                   check=True)
    return str(lib)


def test_battery_passes_on_the_oracle_itself():
    for name, f, kw in battery():
        f(**kw)


@pytest.mark.parametrize("name,subs", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, subs):
    lib = build_mutant(tmp_path, subs)
    caught = None
    with oracle.oracle.use_library(lib):
        for pin, f, kw in battery():
            try:
                f(**kw)
            except Exception as e:        # an assertion, or a check the mutant trips
                caught = (pin, type(e).__name__)
                break
    assert caught is not None, f"no pin catches: {name}"
