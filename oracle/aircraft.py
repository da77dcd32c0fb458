"""Oracle: the auxiliary problems Pi'_1, Pi'_2 of the aircraft mission --
TEST INFRASTRUCTURE ONLY.

Builds, from a scenario of `synth.aircraft`, the discrete abstraction of
Sect. V-B (enclosures from aircraft.c) and the problem data of Sect. VI-A
written out from their definitions:
  - G'_1(Omega) = 0 if the cell lies inside a target box, else infinite;
  - a cell meeting an obstacle box is an avoid state (the running cost of
    any transition into it is infinite);
  - F'(Omega, u) = the cells met by the enclosure of the attainable set;
    a pair whose enclosure leaves the grid on x1, x2 or the speed has an
    infinite cost (its successors leave the operating range);
  - g'_1 = tau + u2^2 (u2 in radians) per transition, as float32;
  - g'_2 = the reward cost for a transition into a cell inside a reward
    box, else g'_1, and G'_2 = V'_1.
Cell bounds are rationals; set membership uses exact integer arithmetic.

Parity status: the enclosures are pinned against independent integrations
of the ODE and closed-form solutions (tests/test_oracle_aircraft.py); the
set membership is pinned by a brute-force check on exact cell corners.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from synth import Problem
from . import lib

AXIS_DEG = (-180, 180)


def table(scn, mass=None) -> np.ndarray:
    """The enclosure table [N4, N3, K, 8] int32 of aircraft.c."""
    N1, N2, N3, N4 = scn.dims
    dims = np.array(scn.dims, dtype=np.int32)
    out = np.zeros(N4 * N3 * scn.K * 8, dtype=np.int32)
    failed = lib().oracle_ac_table(dims.ctypes.data, float(scn.x_max[0]), float(scn.x_max[1]),
                                   float(scn.v_range[0]), float(scn.v_range[1]),
                                   float(scn.mass if mass is None else mass), scn.p_D, scn.p_L, scn.tau,
                                   scn.steps, scn.n_thrust, scn.n_bank, scn.thrust_max, scn.bank_max_deg,
                                   out.ctypes.data)
    if failed:
        raise RuntimeError(f"{failed} enclosures without an a priori enclosure")
    return out.reshape(N4, N3, scn.K, 8)


def bank_rad(scn, b: int) -> float:
    return lib().oracle_ac_bank_rad(b, scn.n_bank, scn.bank_max_deg)


def pair_cost(scn) -> np.ndarray:
    """g'_1 per input: tau + u2 * u2 in double, rounded to float32."""
    out = []
    for u in range(scn.K):
        b = bank_rad(scn, u % scn.n_bank)
        out.append(np.float32(scn.tau + b * b))
    return np.array(out, dtype=np.float32)


def sampled_residual(scn, T, V, G, avoid, reward, states) -> int:
    """Number of sampled states x whose value differs from the backup
    min(G(x), min_u g + max_y ...) computed here from the table (the fixed
    point of Algorithm 1 holds at every state), float32 arithmetic as in
    `problem`."""
    N1, N2, N3, N4 = scn.dims
    gu = pair_cost(scn)
    inf = np.float32(np.inf)
    bad = 0
    for x in np.asarray(states, dtype=np.int64):
        if avoid[x]:
            bad += int(V[x] != inf)
            continue
        i1, i2, i3, i4 = x % N1, (x // N1) % N2, (x // (N1 * N2)) % N3, x // (N1 * N2 * N3)
        best = np.float32(G[x])
        for u in range(scn.K):
            e = T[i4, i3, u]
            n3 = min(int(e[5] - e[4] + 1), N3)
            if not (i1 + e[0] >= 0 and i1 + e[1] < N1 and i2 + e[2] >= 0 and i2 + e[3] < N2 and e[6] >= 0
                    and e[7] < N4 and e[0] <= e[1] and e[2] <= e[3] and n3 > 0):
                continue
            ys = [int(b1 + N1 * (b2 + N2 * (b3 % N3 + N3 * b4)))
                  for b4 in range(e[6], e[7] + 1) for b3 in range(e[4], e[4] + n3)
                  for b2 in range(i2 + e[2], i2 + e[3] + 1) for b1 in range(i1 + e[0], i1 + e[1] + 1)]
            if scn.stage == 2:
                m = max(np.float32(np.float32(scn.reward_cost if reward[y] else gu[u]) + np.float32(V[y]))
                        for y in ys)
                d = np.float32(np.float32(0) + m)
            else:
                d = np.float32(gu[u] + max(np.float32(V[y]) for y in ys))
            if d < best:
                best = d
        bad += int(best != np.float32(V[x]))
    return bad


def _axes(scn):
    """(A, B) of each axis: the cell range [A, B] split into N cells."""
    return ((0, scn.x_max[0]), (0, scn.x_max[1]), AXIS_DEG, tuple(scn.v_range))


def _cell_bounds(A, B, N, i):
    w = Fraction(B - A, N)
    return A + i * w, A + (i + 1) * w


def axis_masks(scn, box, inside: bool):
    """Per axis a boolean array over cell indices: the cell lies inside
    [lo, hi] (inside=True) or meets it."""
    out = []
    for a, (A, B) in enumerate(_axes(scn)):
        lo, hi = box[0][a], box[1][a]
        m = np.zeros(scn.dims[a], dtype=bool)
        for i in range(scn.dims[a]):
            c0, c1 = _cell_bounds(A, B, scn.dims[a], i)
            m[i] = (c0 >= lo and c1 <= hi) if inside else (c0 <= hi and c1 >= lo)
        out.append(m)
    return out


def cell_set(scn, boxes, inside: bool) -> np.ndarray:
    """[n] bool over linear cell ids x = i1 + N1 (i2 + N2 (i3 + N3 i4))."""
    N1, N2, N3, N4 = scn.dims
    res = np.zeros((N4, N3, N2, N1), dtype=bool)
    for box in boxes:
        m = axis_masks(scn, box, inside)
        res |= m[3][:, None, None, None] & m[2][None, :, None, None] & m[1][None, None, :, None] & \
            m[0][None, None, None, :]
    return res.reshape(-1)


def problem(scn, T=None, G=None) -> Problem:
    """The problem Pi'_stage as explicit successor lists (float32 costs).
    Stage 2 puts the whole running cost on the transitions (pair part 0)
    and takes G (e.g. V'_1) as its terminal cost."""
    N1, N2, N3, N4 = scn.dims
    K = scn.K
    n = scn.n
    if T is None:
        T = table(scn)
    target = cell_set(scn, scn.target, True)
    avoid = cell_set(scn, scn.avoid, False)
    reward = cell_set(scn, scn.reward, True) if scn.reward else np.zeros(n, dtype=bool)
    gu = pair_cost(scn)
    inf = np.float32(np.inf)
    # per pair (id p = x K + u): its table entry and the ranges of its box
    p = np.arange(n * K, dtype=np.int64)
    x, u = p // K, p % K
    i1, i2 = x % N1, (x // N1) % N2
    i3, i4 = (x // (N1 * N2)) % N3, x // (N1 * N2 * N3)
    e = T[i4, i3, u].astype(np.int64)   # [nK, 8]
    lo1, lo2, lo3, lo4 = i1 + e[:, 0], i2 + e[:, 2], e[:, 4], e[:, 6]
    n1, n2 = e[:, 1] - e[:, 0] + 1, e[:, 3] - e[:, 2] + 1
    n3, n4 = np.minimum(e[:, 5] - e[:, 4] + 1, N3), e[:, 7] - e[:, 6] + 1
    valid = (lo1 >= 0) & (i1 + e[:, 1] < N1) & (lo2 >= 0) & (i2 + e[:, 3] < N2) & (lo4 >= 0) & \
        (e[:, 7] < N4) & (n1 > 0) & (n2 > 0) & (n3 > 0) & (n4 > 0)
    gp = np.where(valid, gu[u] if scn.stage == 1 else np.float32(0), inf).astype(np.float32)
    # rows: the box's cells, speed outermost and x1 innermost, the heading
    # taken mod N3; a pair of infinite cost keeps the row {x}
    lens = np.where(valid, n1 * n2 * n3 * n4, 1)
    ptr = np.zeros(n * K + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(lens)
    idx = np.empty(int(ptr[-1]), dtype=np.int32)
    idx[ptr[:-1][~valid]] = x[~valid]
    v = np.nonzero(valid)[0]
    m1, m2, m3, m4 = (int(a[v].max()) if v.size else 0 for a in (n1, n2, n3, n4))
    for t4 in range(m4):
        for t3 in range(m3):
            for t2 in range(m2):
                for t1 in range(m1):
                    w = v[(t1 < n1[v]) & (t2 < n2[v]) & (t3 < n3[v]) & (t4 < n4[v])]
                    pos = ptr[w] + ((t4 * n3[w] + t3) * n2[w] + t2) * n1[w] + t1
                    idx[pos] = (lo1[w] + t1) + N1 * ((lo2[w] + t2) + N2 * ((lo3[w] + t3) % N3 + N3 * (lo4[w] + t4)))
    g_edge = None
    if scn.stage == 2:
        src_u = np.repeat(np.arange(n * K, dtype=np.int64) % K, lens)
        g_edge = np.where(reward[idx], np.float32(scn.reward_cost), gu[src_u]).astype(np.float32)
    Gv = np.where(target, np.float32(0), inf).astype(np.float32) if G is None else np.asarray(G, np.float32)
    return Problem(dims=tuple(scn.dims), ndim=4, K=K, dtype="f32", G=Gv, g=gp, avoid=avoid.astype(np.uint8),
                   succ_ptr=ptr, succ_idx=idx, target=target, name=scn.name, g_edge=g_edge)
