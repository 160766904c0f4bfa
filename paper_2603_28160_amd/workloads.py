"""Seeded synthetic workloads for the milling-topography simulator.

This module only describes inputs: tool, cut and grid parameter records, and the seeded
random draws that produce them.  It holds none of the method's arithmetic, so both the GPU
library binding and the CPU oracle can take their inputs from it.

Shapes follow the paper's face-milling workloads (Sec. 4.2, 4.3: a D = 10 mm class tool,
2-4 teeth, feed per tooth 0.02-0.6 mm, micrometre-scale runout) and extend them with the
ball-end, helix, tilt, variable-pitch and raster-pass tools of the benchmark configurations.
Lengths are in mm and angles in rad.  Random numbers come from numpy's PCG64 generator seeded
with 28160 + configuration number (plus the simulation index inside a batch).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

ROUND = 0   # round cutting edge: circular insert / corner-radius profile (Eq. (1))
BALL = 1    # ball end

SEED_BASE = 28160


@dataclass
class Tool:
    kind: int
    n_teeth: int
    n_edge: int
    D: float
    R_edge: float = 0.0
    helix: float = 0.0
    rake_radial: float = 0.0
    rake_axial: float = 0.0
    theta: Optional[Tuple[float, ...]] = None   # tooth angles; None = uniform pitch
    runout_ecc: float = 0.0
    runout_phase: float = 0.0
    eps_r: Tuple[float, ...] = ()                # per-insert radial offsets
    eps_a: Tuple[float, ...] = ()                # per-insert axial offsets
    tilt_lead: float = 0.0
    tilt_side: float = 0.0


@dataclass
class Cut:
    f_z: float
    a_p: float
    a_e: float = 0.0
    phi0: float = 0.0
    steps_per_rev: int = 360
    n_passes: int = 0          # 0: auto
    n_steps: int = 0           # steps per pass, 0: auto
    x_start: float = math.nan  # NaN: auto
    y_first: float = math.nan  # NaN: auto
    time_mode: int = 0         # 0: steps_per_rev steps per revolution; 1: fixed time step dt
    v_c: float = math.nan      # cutting speed, m/min (time_mode 1)
    dt: float = math.nan       # time step, s (time_mode 1)
    x_end: float = math.nan    # end of travel for the automatic step count; NaN: auto


@dataclass
class Grid:
    x0: float
    y0: float
    dd: float
    nx: int
    ny: int


@dataclass
class Sim:
    tool: Tool
    cut: Cut
    grid: Grid
    name: str = ""

    def replace(self, **kw) -> "Sim":
        return dataclasses.replace(self, **kw)


def centred_grid(nx: int, ny: int, dd: float, cx: float = 0.0, cy: float = 0.0) -> Grid:
    """Grid of nx x ny nodes spaced dd whose node block is centred on (cx, cy)."""
    return Grid(x0=cx - 0.5 * (nx - 1) * dd, y0=cy - 0.5 * (ny - 1) * dd, dd=dd, nx=nx, ny=ny)


def _rng(config: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE + config, index])


# --- configuration 1: plain FP64 single pass -----------------------------------------------

def config1() -> Sim:
    """Round-edge ("flat") mill D = 10 mm, 2 flutes, helix 30 deg, 5 um runout at a seeded
    phase, f_z = 0.1 mm, 360 steps/rev, 20 edge points, one straight pass, a_p = 0.5 mm;
    1 x 1 mm Z-map at 5 um (200 x 200)."""
    r = _rng(1)
    tool = Tool(kind=ROUND, n_teeth=2, n_edge=20, D=10.0, R_edge=5.0,
                helix=math.radians(30.0), runout_ecc=0.005,
                runout_phase=float(r.uniform(0.0, 2.0 * math.pi)))
    cut = Cut(f_z=0.1, a_p=0.5, steps_per_rev=360, n_passes=1, y_first=0.0)
    return Sim(tool, cut, centred_grid(200, 200, 0.005), name="config1_flat_d10_200x200_f64")


# --- configuration 2: ball-end raster ---------------------------------------------------------

def config2(nx: int = 5000, ny: int = 5000, dd: float = 0.001) -> Sim:
    """Ball end R = 3 mm, 4 flutes, helix 30 deg, lead tilt 15 deg, runout U(0, 8) um at a
    seeded phase, f_z = 0.08 mm, stepover 0.3 mm parallel passes, 720 steps/rev, 64 edge
    points, a_p = 0.5 mm; 5 x 5 mm at 1 um (5000 x 5000)."""
    r = _rng(2)
    ecc = float(r.uniform(0.0, 0.008))
    phase = float(r.uniform(0.0, 2.0 * math.pi))
    tool = Tool(kind=BALL, n_teeth=4, n_edge=64, D=6.0, helix=math.radians(30.0),
                runout_ecc=ecc, runout_phase=phase, tilt_lead=math.radians(15.0))
    cut = Cut(f_z=0.08, a_p=0.5, a_e=0.3, steps_per_rev=720)
    return Sim(tool, cut, centred_grid(nx, ny, dd), name=f"config2_ball_r3_{nx}x{ny}")


# --- configuration 3: batch of uneven simulations ---------------------------------------------

def random_sim(config: int, index: int, side_max: int = 2048, n_edge: int = 64,
               steps_per_rev: int = 720) -> Sim:
    """One seeded simulation of the batch/serving mix: tool type round/ball 50/50,
    D ~ U(4, 16) mm, flutes in {2, 3, 4}, helix ~ U(20, 45) deg, f_z ~ U(0.02, 0.2) mm,
    stepover ~ U(0.1, 1.0) mm, runout ~ U(0, 10) um at phase ~ U(0, 2 pi), lead tilt
    ~ U(0, 30) deg, square grid with side ~ U{256..side_max} cells at dd ~ U(1, 5) um."""
    r = _rng(config, index)
    kind = BALL if r.uniform() < 0.5 else ROUND
    D = float(r.uniform(4.0, 16.0))
    z_n = int(r.integers(2, 5))
    helix = math.radians(float(r.uniform(20.0, 45.0)))
    f_z = float(r.uniform(0.02, 0.2))
    a_e = float(r.uniform(0.1, 1.0))
    ecc = float(r.uniform(0.0, 0.010))
    phase = float(r.uniform(0.0, 2.0 * math.pi))
    tilt = math.radians(float(r.uniform(0.0, 30.0)))
    side = int(r.integers(256, side_max + 1))
    dd = float(r.uniform(0.001, 0.005))
    tool = Tool(kind=kind, n_teeth=z_n, n_edge=n_edge, D=D,
                R_edge=0.5 * D if kind == ROUND else 0.0, helix=helix,
                runout_ecc=ecc, runout_phase=phase, tilt_lead=tilt)
    cut = Cut(f_z=f_z, a_p=0.5, a_e=a_e, steps_per_rev=steps_per_rev)
    return Sim(tool, cut, centred_grid(side, side, dd), name=f"mix{config}_{index}")


def config3(n: int = 256) -> List[Sim]:
    """Batch of n seeded simulations (grid sides up to 2048)."""
    return [random_sim(3, i, side_max=2048) for i in range(n)]


def config4_requests(n: int, rate: float, seed_offset: int = 0) -> List[Tuple[float, Sim]]:
    """Serving workload: n requests drawn like configuration 3 with sides up to 4096 and
    Poisson arrivals at `rate` requests/s.  Returns (arrival time in s, simulation) pairs."""
    r = _rng(4, 1_000_000 + seed_offset)
    gaps = r.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    return [(float(t[i]), random_sim(4, seed_offset * 1_000_003 + i, side_max=4096))
            for i in range(n)]


# --- configuration 5: one large field ---------------------------------------------------------

def config5(nx: int = 40000, ny: int = 40000, dd: float = 0.0005) -> Sim:
    """Round-edge mill D = 12 mm, 4 flutes at 0/88/180/268 deg (pitch 88/92/88/92),
    helix 35 deg, runout 6 um at a seeded phase, lead tilt 5 deg, f_z = 0.12 mm, stepover
    2 mm, 720 steps/rev, 128 edge points, a_p = 0.5 mm; 20 x 20 mm at 0.5 um."""
    r = _rng(5)
    tool = Tool(kind=ROUND, n_teeth=4, n_edge=128, D=12.0, R_edge=6.0,
                helix=math.radians(35.0),
                theta=tuple(math.radians(a) for a in (0.0, 88.0, 180.0, 268.0)),
                runout_ecc=0.006, runout_phase=float(r.uniform(0.0, 2.0 * math.pi)),
                tilt_lead=math.radians(5.0))
    cut = Cut(f_z=0.12, a_p=0.5, a_e=2.0, steps_per_rev=720)
    return Sim(tool, cut, centred_grid(nx, ny, dd), name=f"config5_flat_d12_{nx}x{ny}")


# --- the paper's own tool (Case 2, Sec. 4.2) ----------------------------------------------------

def paper_case2_tool(eps_r: float = 0.0, eps_a: float = 0.0, n_edge: int = 40) -> Tool:
    """Face mill D = 10 mm with 2 round inserts of radius 5 mm, radial rake 0.6 deg, axial
    rake 0 deg (tool table of Sec. 4.2); insert K carries the runout (K-1)*eps (Eq. (2))."""
    return Tool(kind=ROUND, n_teeth=2, n_edge=n_edge, D=10.0, R_edge=5.0,
                rake_radial=math.radians(0.6), rake_axial=0.0,
                eps_r=(0.0, eps_r), eps_a=(0.0, eps_a))


# --- the paper's computational-performance conditions (Sec. 4.3) -------------------------------

# (number, v_c m/min, f_z mm/tooth, a_p mm) of the paper's table of selected milling parameters
PAPER_CONDITIONS = ((1, 170, 0.4, 0.3), (2, 170, 0.5, 0.4), (3, 170, 0.6, 0.5),
                    (4, 200, 0.4, 0.3), (5, 200, 0.5, 0.4), (6, 200, 0.6, 0.5),
                    (7, 230, 0.4, 0.3), (8, 230, 0.5, 0.4), (9, 230, 0.6, 0.5))
PAPER_DT = 0.4e-6          # s: the time step that reproduces the paper's trajectory-point counts


def paper_mode(no: int, dd: float = 0.005, n_edge: int = 40, travel: float = 10.0) -> Sim:
    """Condition `no` of the paper's performance study: the Case-2 tool without runout, one
    straight pass along the 10 mm length of a 10 x 5 mm surface at the paper's fixed time step,
    the surface sampled at dd (the paper does not state its grid; 5 um by default)."""
    _, vc, fz, ap = PAPER_CONDITIONS[no - 1]
    tool = paper_case2_tool(n_edge=n_edge)
    nx, ny = int(round(10.0 / dd)), int(round(5.0 / dd))
    grid = centred_grid(nx, ny, dd)
    x_lo = grid.x0 - 0.5 * dd
    cut = Cut(f_z=fz, a_p=ap, n_passes=1, y_first=0.0, time_mode=1, v_c=float(vc), dt=PAPER_DT,
              x_start=x_lo, x_end=x_lo + travel)
    return Sim(tool, cut, grid, name=f"paper_condition{no}_{nx}x{ny}")


# --- dataset generation (Sec. 4.3: many simulations over parameter ranges by LHS) ------------

DATASET_RANGES = {
    "D": (4.0, 16.0), "n_teeth": (2.0, 5.0), "helix": (math.radians(20.0), math.radians(45.0)),
    "f_z": (0.02, 0.2), "a_e": (0.1, 1.0), "runout_ecc": (0.0, 0.010),
    "runout_phase": (0.0, 2.0 * math.pi), "tilt_lead": (0.0, math.radians(30.0)),
}


def lhs(n: int, ranges, seed: int = 0) -> List[dict]:
    """Latin hypercube sample of n points in the box `ranges` (name -> (lo, hi)): every
    parameter's range is cut into n equal strata, each stratum holds exactly one point at a
    uniform position inside it, and the strata are paired across parameters by independent
    random permutations."""
    r = _rng(6, seed)
    out = [dict() for _ in range(n)]
    for name, (lo, hi) in ranges.items():
        u = (r.permutation(n) + r.random(n)) / n
        for k in range(n):
            out[k][name] = lo + (hi - lo) * float(u[k])
    return out


def dataset_sims(n: int, kind: int = BALL, side: int = 1024, dd: float = 0.002,
                 seed: int = 0, ranges=None) -> List[Sim]:
    """n simulations of one tool type over the parameter box (DATASET_RANGES by default) drawn
    by Latin hypercube sampling, all on the same side x side grid at dd, so that the Z-maps
    stack into one dataset tensor.  The flute count takes the integer part of its stratum."""
    sims = []
    for k, p in enumerate(lhs(n, ranges or DATASET_RANGES, seed)):
        D = p["D"]
        tool = Tool(kind=kind, n_teeth=min(4, int(p["n_teeth"])), n_edge=64, D=D,
                    R_edge=0.5 * D if kind == ROUND else 0.0, helix=p["helix"],
                    runout_ecc=p["runout_ecc"], runout_phase=p["runout_phase"],
                    tilt_lead=p["tilt_lead"])
        cut = Cut(f_z=p["f_z"], a_p=0.5, a_e=p["a_e"], steps_per_rev=720)
        sims.append(Sim(tool, cut, centred_grid(side, side, dd), name=f"lhs{seed}_{k}"))
    return sims


def synthetic_surface(nx: int, ny: int, dd: float, seed: int = 0, hole_frac: float = 0.0,
                      feed: float = 0.1, depth: float = 0.002) -> np.ndarray:
    """Seeded stand-in for a milled Z-map, [ny, nx] float64 in mm: feed marks along x (a
    cosine of wavelength `feed` and amplitude `depth`), waviness along y (wavelength 1.3 mm),
    a tilted plane, white noise of depth/20, and holes (+inf) at a fraction hole_frac of the
    cells.  Input for the surface-texture operators; it holds none of the method."""
    r = _rng(7, seed)
    x = np.arange(nx) * dd
    y = np.arange(ny) * dd
    X, Y = np.meshgrid(x, y)
    ph = r.uniform(0.0, 2.0 * math.pi, 2)
    Z = (-0.5 + depth * np.cos(2.0 * math.pi * X / feed + ph[0])
         + 0.25 * depth * np.cos(2.0 * math.pi * Y / 1.3 + ph[1])
         + float(r.uniform(-0.01, 0.01)) * X + float(r.uniform(-0.01, 0.01)) * Y
         + r.normal(0.0, depth / 20.0, (ny, nx)))
    if hole_frac > 0.0:
        Z[r.random((ny, nx)) < hole_frac] = np.inf
    return Z


CONFIGS = {1: config1, 2: config2, 5: config5}
