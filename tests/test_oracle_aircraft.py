"""Pins of the oracle's aircraft abstraction (oracle/aircraft.c, oracle/aircraft.py)
against facts that do not come from the oracle itself:

* sin and cos of the enclosures against the C library, and the reduction
  constants against a decimal expansion of pi;
* enclosures of the attainable sets (Sect. V-B) against trajectories of the
  aircraft ODE (Sect. VI-A) integrated independently by scipy's DOP853;
* closed-form solutions of the ODE for level flight (bank angle 0);
* the table's cell ranges against the cells of sampled end points;
* the cell sets against the definitions with exact rationals;
* planted mistakes in aircraft.c (a dropped drag term, a wrong sign, the
  wrong trigonometric function) fail the containment pin.
"""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import oracle.aircraft as OA
import synth.aircraft as SA

PAPER = dict(mass=4250.0, p_D=1.8, p_L=85.0, tau=0.45)


def field(t, x, u1, u2, mass, p_D, p_L):
    """Sect. VI-A, the point-mass aircraft."""
    return [x[3] * math.cos(x[2]), x[3] * math.sin(x[2]), p_L * x[3] * math.sin(u2) / mass,
            (u1 - p_D * x[3] ** 2) / mass]


def flow(x0, u1, u2, tau=0.45, mass=4250.0, p_D=1.8, p_L=85.0):
    sol = solve_ivp(field, (0.0, tau), list(x0), method="DOP853", rtol=1e-12, atol=1e-12,
                    args=(u1, u2, mass, p_D, p_L))
    return sol.y[:, -1]


def enclose(lo, hi, u1, u2, steps=4, L=None, **kw):
    prm = dict(PAPER, **kw)
    L = L or oracle.lib()
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    olo, ohi = np.zeros(4), np.zeros(4)
    rc = L.oracle_ac_enclose(lo.ctypes.data, hi.ctypes.data, u1, u2, prm["mass"], prm["p_D"], prm["p_L"],
                             prm["tau"], steps, olo.ctypes.data, ohi.ctypes.data)
    assert rc == 0
    return olo, ohi


def test_trig_against_libm():
    L = oracle.lib()
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-16, 16, 20000), np.linspace(-7, 7, 2001),
                         [0.0, math.pi / 2, -math.pi, math.pi, 1e-300, -1e-300]])
    err = max(max(abs(L.oracle_ac_sin(float(x)) - math.sin(x)), abs(L.oracle_ac_cos(float(x)) - math.cos(x)))
              for x in xs)
    # the enclosures widen every value by 1e-14; the evaluation must stay well inside
    assert err < 1e-15


def test_reduction_constants_from_pi():
    """pi/2 = head + tail: head is pi/2 cut to 33 significant bits, tail the
    double nearest the rest; the double just below pi is the nearest double."""
    getcontext().prec = 60
    pi = Decimal("3.14159265358979323846264338327950288419716939937510582097494459")
    src = oracle.source("aircraft")

    def const(name):
        line = next(ln for ln in src.splitlines() if ln.startswith(f"#define {name} "))
        return float(line.split()[2])

    head, tail = const("AC_PIO2_A"), const("AC_PIO2_B")
    assert Decimal(head) == (pi / 2 * 2 ** 32).to_integral_value(rounding="ROUND_FLOOR") / Decimal(2) ** 32
    assert tail == float(pi / 2 - Decimal(head))
    assert const("AC_PI_DN") == float(pi) and Decimal(const("AC_PI_DN")) < pi
    assert const("AC_2_OVER_PI") == float(2 / pi)


def _random_boxes(rng, count):
    for _ in range(count):
        lo = np.array([0.0, 0.0, rng.uniform(-math.pi, math.pi), rng.uniform(50, 84)])
        w = np.array([12.5, 800 / 70, 2 * math.pi / 75, 35 / 135]) * rng.uniform(0.3, 2.0, 4)
        yield lo, lo + w


def test_enclosure_contains_trajectories():
    rng = np.random.default_rng(2)
    for k, (lo, hi) in enumerate(_random_boxes(rng, 40)):
        u1 = [0.0, 4500.0, 9000.0, 13500.0, 18000.0][k % 5]
        u2 = math.radians([-40.0, -13.3, 0.0, 26.7, 40.0][k % 5 if k % 3 else 2])
        olo, ohi = enclose(lo, hi, u1, u2)
        pts = [lo + (hi - lo) * rng.uniform(0, 1, 4) for _ in range(12)]
        pts += [np.where([(c >> a) & 1 for a in range(4)], hi, lo) for c in range(16)]
        for p in pts:
            y = flow(p, u1, u2)
            assert np.all(y >= olo - 1e-9) and np.all(y <= ohi + 1e-9), (k, p, y, olo, ohi)


def test_enclosure_is_tight():
    """The enclosure is not much wider than the spread of the end points
    (first order in the sampling time: at most a few times the cell)."""
    rng = np.random.default_rng(3)
    for lo, hi in _random_boxes(rng, 10):
        olo, ohi = enclose(lo, hi, 9000.0, math.radians(13.3))
        ys = np.array([flow(lo + (hi - lo) * rng.uniform(0, 1, 4), 9000.0, math.radians(13.3)) for _ in range(40)])
        spread = ys.max(0) - ys.min(0)
        assert np.all(ohi - olo <= 2.0 * (hi - lo) + 2.0 * spread + 1e-6)


@pytest.mark.parametrize("u1", [0.0, 4500.0, 13500.0, 18000.0])
def test_level_flight_closed_form(u1):
    """Bank angle 0: the heading stays, x4' = (u1 - p_D x4^2) / m is a
    Riccati equation with the closed form below, and x1, x2 follow from
    integrating x4 along the fixed heading."""
    m, pD, tau = 4250.0, 1.8, 0.45
    for x3 in (0.0, 0.7, -2.5, 3.0):
        for v0 in (50.0, 66.0, 84.0):
            olo, ohi = enclose([0, 0, x3, v0], [0, 0, x3, v0], u1, 0.0)
            b = pD / m
            if u1 == 0:
                v = v0 / (1 + b * v0 * tau)
                s = math.log(1 + b * v0 * tau) / b
            else:
                a = u1 / m
                r = math.sqrt(a / b)
                k = math.sqrt(a * b)
                if abs(v0 - r) < 1e-12:  # the equilibrium speed
                    v, s = v0, v0 * tau
                elif v0 < r:
                    c = math.atanh(v0 / r)
                    v = r * math.tanh(k * tau + c)
                    s = (math.log(math.cosh(k * tau + c)) - math.log(math.cosh(c))) / b
                else:
                    c = math.atanh(r / v0)
                    v = r / math.tanh(k * tau + c)
                    s = (math.log(math.sinh(k * tau + c)) - math.log(math.sinh(c))) / b
            exact = np.array([s * math.cos(x3), s * math.sin(x3), x3, v])
            assert np.all(olo <= exact + 1e-9) and np.all(exact <= ohi + 1e-9), (x3, v0, olo, exact, ohi)
            assert np.all(ohi - olo < np.array([2.0, 2.0, 1e-9, 0.05]))


def test_table_contains_sampled_cells():
    """Every entry's cell ranges hold the cells where sampled trajectories
    from the entry's cell end (x1, x2 relative to the cell at the origin)."""
    scn = SA.small(1)
    T = OA.table(scn)
    N1, N2, N3, N4 = scn.dims
    eta = np.array([scn.x_max[0] / N1, scn.x_max[1] / N2, 2 * math.pi / N3, 35.0 / N4])
    rng = np.random.default_rng(4)
    for _ in range(150):
        i3, i4, u = int(rng.integers(N3)), int(rng.integers(N4)), int(rng.integers(scn.K))
        u1 = OA.lib().oracle_ac_thrust(u // scn.n_bank, scn.n_thrust, scn.thrust_max)
        u2 = OA.bank_rad(scn, u % scn.n_bank)
        lo = np.array([0.0, 0.0, -math.pi + i3 * eta[2], 50 + i4 * eta[3]])
        e = T[i4, i3, u]
        for _ in range(4):
            y = flow(lo + eta * rng.uniform(0, 1, 4), u1, u2, mass=scn.mass)
            c = np.floor((y - np.array([0, 0, -math.pi, 50])) / eta).astype(int)
            assert e[0] <= c[0] <= e[1] and e[2] <= c[1] <= e[3], (e, c)
            assert e[4] <= c[2] <= e[5] or e[4] <= c[2] + N3 <= e[5] or e[4] <= c[2] - N3 <= e[5], (e, c)
            if 0 <= c[3] < N4:
                assert e[6] <= c[3] <= e[7], (e, c)


def test_cell_sets_exact():
    scn = SA.small(2)
    axes = ((0, scn.x_max[0]), (0, scn.x_max[1]), (-180, 180), tuple(scn.v_range))
    for boxes, inside in ((scn.target, True), (scn.avoid, False), (scn.reward, True)):
        got = OA.cell_set(scn, boxes, inside).reshape(scn.dims[::-1])
        rng = np.random.default_rng(5)
        for _ in range(300):
            c = [int(rng.integers(d)) for d in scn.dims]
            want = False
            for lo, hi in boxes:
                ok = True
                for a in range(4):
                    A, B = axes[a]
                    c0 = A + Fraction(c[a] * (B - A), scn.dims[a])
                    c1 = A + Fraction((c[a] + 1) * (B - A), scn.dims[a])
                    ok &= (lo[a] <= c0 and c1 <= hi[a]) if inside else not (c1 < lo[a] or c0 > hi[a])
                want |= ok
            assert got[c[3], c[2], c[1], c[0]] == want


def test_small_problem_solves_to_a_fixed_point():
    scn = SA.small(1)
    T = OA.table(scn)
    P = OA.problem(scn, T)
    r = oracle.solve(P, precision="f32")
    V = r["V"]
    assert r["status"] == oracle.OK and r["residual"] == 0
    assert np.all(V[P.target & (P.avoid == 0)] == 0)
    assert np.isfinite(V).sum() > P.target.sum()
    states = np.random.default_rng(6).integers(0, scn.n, 300)
    assert OA.sampled_residual(scn, T, V, P.G, P.avoid, np.zeros(scn.n, bool), states) == 0
    # the second problem: reward for transitions into the fire at drop speed
    scn2 = SA.small(2)
    P2 = OA.problem(scn2, G=V)
    r2 = oracle.solve(P2, precision="f32")
    assert r2["status"] == oracle.OK and r2["residual"] == 0
    reward = OA.cell_set(scn2, scn2.reward, True)
    assert OA.sampled_residual(scn2, OA.table(scn2), r2["V"], P2.G, P2.avoid, reward, states) == 0
    assert np.all(r2["V"] <= P2.G)


MUTANTS = {
    "drag dropped": ("ac_scale(ac_sqr(x[3]), in->p_D)", "ac_scale(ac_sqr(x[3]), 0.0)"),
    "sign of x2 rate": ("f[1] = ac_mul(x[3], s);", "f[1] = ac_mul(x[3], ac_sub(ac_pt(0.0), s));"),
    "cos for sin": ("f[1] = ac_mul(x[3], s);", "f[1] = ac_mul(x[3], c);"),
    "half step": ("X[a].lo = y.lo > B[a].lo ? y.lo : B[a].lo;",
                  "y = ac_add(X[a], ac_scale(f[a], 0.5 * h));\n                X[a].lo = y.lo > B[a].lo ? y.lo : B[a].lo;"),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_containment_pin_catches_planted_mistakes(mutant, tmp_path):
    old, new = MUTANTS[mutant]
    src = oracle.source("aircraft")
    assert old in src
    path = oracle.build_variant(src.replace(old, new, 1), str(tmp_path / "liboracle_ac.so"), which="aircraft")
    with oracle.use_variant(path):
        L = oracle.lib()
        rng = np.random.default_rng(7)
        caught = False
        for k, (lo, hi) in enumerate(_random_boxes(rng, 12)):
            u1, u2 = [0.0, 18000.0, 9000.0][k % 3], math.radians([-40.0, 40.0, 26.7][k % 3])
            olo, ohi = enclose(lo, hi, u1, u2, L=L)
            for c in range(16):
                y = flow(np.where([(c >> a) & 1 for a in range(4)], hi, lo), u1, u2)
                caught |= bool(np.any(y < olo - 1e-9) or np.any(y > ohi + 1e-9))
        assert caught, mutant


def test_closed_loop_keeps_the_guarantee():
    """The method's guarantee (Sect. V-B with the theorem on Algorithm 1):
    the controller of the abstraction, applied to the real aircraft (its ODE
    integrated independently, the input held for tau and chosen from the
    cell the state is in), keeps it inside the area and off the obstacles
    and reaches the target with an accumulated cost of at most V(x0).  An
    enclosure that misses part of an attainable set would break this."""
    scn = SA.small(1)
    P = OA.problem(scn)
    r = oracle.solve(P, precision="f32")
    V, pol = r["V"], r["policy"]
    N1, N2, N3, N4 = scn.dims
    eta = np.array([scn.x_max[0] / N1, scn.x_max[1] / N2, 2 * math.pi / N3, 35.0 / N4])
    lo = np.array([0.0, 0.0, -math.pi, 50.0])
    gu = OA.pair_cost(scn)
    rng = np.random.default_rng(8)
    start = np.nonzero(np.isfinite(V) & ~P.target)[0]
    assert start.size > 100
    for x0 in rng.choice(start, 40, replace=False):
        c = np.array([x0 % N1, (x0 // N1) % N2, (x0 // (N1 * N2)) % N3, x0 // (N1 * N2 * N3)])
        s = lo + (c + rng.uniform(0.05, 0.95, 4)) * eta
        cost = 0.0
        for _ in range(400):
            c = np.floor((s - lo) / eta).astype(int)
            assert np.all(c >= 0) and c[0] < N1 and c[1] < N2 and c[3] < N4, ("left the area", x0, s)
            x = int(c[0] + N1 * (c[1] + N2 * (c[2] + N3 * c[3])))
            assert not P.avoid[x], ("obstacle", x0, s)
            if pol[x] == oracle.HANDOVER:
                break
            u = int(pol[x])
            assert u >= 0, ("no controller", x0, x)
            cost += float(gu[u])
            s = flow(s, OA.lib().oracle_ac_thrust(u // scn.n_bank, scn.n_thrust, scn.thrust_max),
                     OA.bank_rad(scn, u % scn.n_bank), mass=scn.mass)
            s[2] = (s[2] + math.pi) % (2 * math.pi) - math.pi
        else:
            raise AssertionError(("target not reached", x0))
        assert P.target[x]
        assert cost <= float(V[x0]) + 1e-4, (x0, cost, V[x0])
