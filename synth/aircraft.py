"""Seeded scenarios for the aircraft abstraction (inputs only).

The aerial firefighting mission of Sect. VI-A: a point-mass aircraft with
positions x1, x2 (metres), heading x3 and speed x4, thrust u1 and bank angle
u2, sampled with tau = 0.45 s.  Problem Pi_1 flies the empty aircraft (mass
m_1) back to the runway; Pi_2 flies the loaded aircraft (m_2) over the fire,
with a reward for every transition into the fire region at drop speed, and
hands over to Pi_1 through G_2 = V_1.

A scenario fixes the grid, the constants of the model, the input grid and
the sets of the specification as closed boxes with integer bounds per axis
(x1 and x2 in metres, the heading in degrees within [-180, 180], the speed in
m/s).  The paper prints the runway, landing, no-fly and drop sets; the hills
and the fire are drawn in a figure only, so here they are seeded rectangles.
Grids other than the paper's scale the sets with the area and widen them to
at least a few cells, so that small grids still have targets.

Nothing here computes any part of the abstraction or of the solver.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

from . import Stream, instance_seed

Box = Tuple[Tuple[int, int, int, int], Tuple[int, int, int, int]]

PAPER_DIMS = (200, 70, 75, 135)
PAPER_AREA = (2500, 800)
MASS_EMPTY = 4250.0
MASS_LOADED = 6250.0
REWARD_COST = float(np.float32(-5 * 0.45))  # -5 tau per transition into the fire at drop speed


@dataclasses.dataclass
class Scenario:
    dims: tuple                  # cells on x1, x2, heading, speed
    x_max: tuple                 # positions in [0, x_max[a]] metres
    v_range: tuple = (50, 85)    # speed range, m/s
    mass: float = MASS_EMPTY
    p_D: float = 1.8
    p_L: float = 85.0
    tau: float = 0.45
    steps: int = 4               # integration steps per sampling period
    n_thrust: int = 5            # thrust grid vertices on [0, thrust_max]
    n_bank: int = 7              # bank-angle grid vertices on [-bank_max, bank_max]
    thrust_max: float = 18000.0
    bank_max_deg: float = 40.0
    target: List[Box] = dataclasses.field(default_factory=list)   # G = 0 on cells inside one
    avoid: List[Box] = dataclasses.field(default_factory=list)    # cells meeting one are obstacles
    reward: List[Box] = dataclasses.field(default_factory=list)   # transitions into cells inside one
    reward_cost: float = REWARD_COST
    stage: int = 1
    name: str = ""

    @property
    def K(self) -> int:
        return self.n_thrust * self.n_bank

    @property
    def n(self) -> int:
        return int(np.prod(self.dims))


def _full(lo12, hi12, head=(-180, 180), speed=(50, 85)) -> Box:
    return ((int(lo12[0]), int(lo12[1]), int(head[0]), int(speed[0])),
            (int(hi12[0]), int(hi12[1]), int(head[1]), int(speed[1])))


def _rect(rng: Stream, X: int, Y: int, wfrac, hfrac, xr, yr):
    """A seeded rectangle: widths as fractions of the area, lower corner in
    the fractional windows xr, yr."""
    u = rng.uniform(4)
    w = int(X * (wfrac[0] + (wfrac[1] - wfrac[0]) * u[0]))
    h = int(Y * (hfrac[0] + (hfrac[1] - hfrac[0]) * u[1]))
    x0 = int(X * (xr[0] + (xr[1] - xr[0]) * u[2]))
    y0 = int(Y * (yr[0] + (yr[1] - yr[0]) * u[3]))
    return (x0, y0), (min(X, x0 + max(w, 1)), min(Y, y0 + max(h, 1)))


def scenario(dims=PAPER_DIMS, x_max=PAPER_AREA, stage: int = 1, seed: int = 0, steps: int = 4,
             cone: int = 0) -> Scenario:
    """Pi_1 (stage 1) or Pi_2 (stage 2) on the grid `dims` over the area
    [0, x_max[0]] x [0, x_max[1]].  On the paper's grid and area the printed
    sets are used as they are.  cone > 0 widens the landing set to headings
    within +-cone degrees at any speed (coarse grids, where the narrow
    landing set is out of worst-case reach)."""
    N1, N2, N3, N4 = dims
    X, Y = x_max
    paper = tuple(dims) == PAPER_DIMS and tuple(x_max) == PAPER_AREA
    wx, wy, wh, wv = X / N1, Y / N2, 360.0 / N3, 35.0 / N4
    if paper:
        rwy = ((300, 100), (900, 180))
        land_h, land_v = 10, 55
        nofly = ((320, 120), (880, 160))
        nofly_h = 12
        drop = (53, 56)
    else:
        x0, y0 = math.floor(0.12 * X), math.floor(0.125 * Y)
        rwy = ((x0, y0), (math.ceil(max(0.36 * X, x0 + 3 * wx)), math.ceil(max(0.225 * Y, y0 + 3 * wy))))
        land_h = math.ceil(max(10.0, 1.01 * wh))
        land_v = 50 + math.ceil(max(5.0, 2.0 * wv))
        nofly = ((math.floor(0.128 * X), math.floor(0.15 * Y)), (math.ceil(0.352 * X), math.ceil(0.2 * Y)))
        nofly_h = land_h + 2
        drop = (53, 53 + math.ceil(max(3.0, 2.0 * wv)))
    if cone:
        land_h, land_v = cone, 85
        nofly_h = cone + 2
    target = [_full(*rwy, head=(-land_h, land_h), speed=(50, land_v))]
    avoid = [_full(*nofly, head=(nofly_h, 180)), _full(*nofly, head=(-180, -nofly_h))]
    sd = instance_seed(2001, seed)
    # hills: west of the runway's end and north of the area's middle, away
    # from the runway and the fire
    for k, (xr, yr) in enumerate((((0.40, 0.48), (0.05, 0.30)), ((0.05, 0.30), (0.55, 0.75)),
                                  ((0.40, 0.50), (0.60, 0.80)))):
        lo, hi = _rect(Stream(sd, k), X, Y, (0.04, 0.08), (0.08, 0.15), xr, yr)
        avoid.append(_full(lo, hi))
    flo, fhi = _rect(Stream(sd, 17), X, Y, (0.06, 0.09), (0.10, 0.16), (0.62, 0.80), (0.45, 0.70))
    fhi = (max(fhi[0], flo[0] + math.ceil(3 * wx)), max(fhi[1], flo[1] + math.ceil(3 * wy)))
    reward = [_full(flo, fhi, speed=drop)] if stage == 2 else []
    return Scenario(dims=tuple(int(d) for d in dims), x_max=(int(X), int(Y)),
                    mass=MASS_EMPTY if stage == 1 else MASS_LOADED, steps=steps, target=target, avoid=avoid,
                    reward=reward, stage=stage,
                    name=f"aircraft_pi{stage}_{'x'.join(map(str, dims))}")


def small(stage: int = 1, seed: int = 0) -> Scenario:
    """A grid the oracle solves in about a second: 16 x 8 cells of 25 m
    over a 400 m x 200 m area, 15-degree heading cells, 16 speed cells,
    landing within 60 degrees of the runway heading."""
    return scenario((16, 8, 24, 16), (400, 200), stage=stage, seed=seed, cone=60)


def medium(stage: int = 1, seed: int = 1) -> Scenario:
    """24 x 12 cells of 25 m over 600 m x 300 m, 15-degree heading cells,
    12 speed cells, landing within 90 degrees (about 83 k cells)."""
    return scenario((24, 12, 24, 12), (600, 300), stage=stage, seed=seed, cone=90)
