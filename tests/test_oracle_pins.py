"""Pins of the CPU oracle to facts other than itself (no GPU).

Each test ties the oracle (Algorithm 1 in C) to: values the paper prints for
its worked example (Fig. 2), brute force from the definitions of Sect. III,
an independent min-max Dijkstra, the textbook Bellman-Ford via scipy for the
ordinary-graph special case, and invariants (fixed-point residual, round and
work bounds of the complexity theorem, the potential-form lower bound).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import brute
from tests import golden_io

INF_I32 = 2**31 - 1


def _pol_name(p, inputs):
    return "U" if p == oracle.HANDOVER else ("none" if p == oracle.NONE else inputs[p])


# ---------------------------------------------------------------- Fig. 2
@pytest.fixture(scope="module")
def fig2():
    return golden_io.load("fig2_example.txt")


def test_fig2_cost_functional(fig2):
    """Example "costs": J = 7, 5, 2 for x and 6, 1 for y (pins the encoding
    of the figure and the cost functional)."""
    prob, inputs, facts = fig2
    b = inputs.index("b")
    sig = {"x": [6, 3, 2, 2, 2], "y": [6, 4, 0, 0, 0]}
    vs = {"v0": [1, 1, 1, 1, 1], "v1": [0, 1, 1, 1, 1], "v2": [0, 0, 1, 1, 1]}
    for traj, v, val in facts["J"]:
        assert brute.cost_J(prob, [b] * 5, vs[v], sig[traj]) == int(val)


def test_fig2_closed_loop_performance(fig2):
    """Example "closed-loop performance": L(7, mu = b) = 2."""
    prob, inputs, facts = fig2
    b = inputs.index("b")
    L = brute.evaluate(prob, [b] * prob.n)
    for st, val in facts["L_all_b"]:
        assert L[int(st) - 1] == int(val)


def test_fig2_oracle_matches_paper(fig2):
    """Example "algorithm": the final controller printed in the paper, both
    as Algorithm 1 leaves it and as the canonical post-pass gives it."""
    prob, inputs, facts = fig2
    r = oracle.solve(prob)
    assert r["status"] == oracle.OK and r["residual"] == 0
    want = {int(s) - 1: name for s, name in facts["mu"]}
    for x, name in want.items():
        assert _pol_name(int(r["mu"][x]), inputs) == name
        assert _pol_name(int(r["policy"][x]), inputs) == name


def test_fig2_frontier_after_round1(fig2):
    """Example "algorithm": after one pass the frontier is X minus {5}."""
    prob, inputs, facts = fig2
    r = oracle.solve(prob, max_rounds=1)
    assert r["status"] == oracle.NEGCYCLE      # cap reached with a non-empty frontier
    want = sorted(int(s) - 1 for s in facts["frontier_after_round1"][0])
    assert sorted(r["frontier"].tolist()) == want


def test_fig2_value_function_brute_force(fig2):
    prob, _, _ = fig2
    r = oracle.solve(prob)
    kl, _ = brute.kleene(prob)
    en = brute.enumerate_V(prob)
    assert r["V"].tolist() == kl == en


def test_fig2_policy_realizes_value(fig2):
    """Theorem on Algorithm 1: mu realizes W (L(., mu) = W)."""
    prob, _, _ = fig2
    r = oracle.solve(prob)
    assert brute.evaluate(prob, r["policy"].tolist()) == r["V"].tolist()
    assert brute.evaluate(prob, r["mu"].tolist()) == r["V"].tolist()


# ---------------------------------------------------------------- negative cycle
def test_negative_cycle_round_cap():
    prob, _, _ = golden_io.load("negcycle.txt")
    r = oracle.solve(prob)
    assert r["status"] == oracle.NEGCYCLE
    assert r["counters"]["rounds"] == prob.n
    with pytest.raises(brute.Diverged):
        brute.kleene(prob)


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(40))
def test_tiny_potential_form_vs_enumeration(seed):
    n = 3 + seed % 4
    K = 2 + seed % 2
    prob = synth.potential_small(1000 + seed, n, K)
    r = oracle.solve(prob)
    assert r["status"] == oracle.OK and r["residual"] == 0
    V = [math.inf if v == INF_I32 else int(v) for v in r["V"]]
    assert V == brute.kleene(prob)[0]
    if K ** n <= 4096:
        assert V == brute.enumerate_V(prob)
    assert [math.inf if v == INF_I32 else v for v in brute.evaluate(prob, r["policy"].tolist())] == V


@pytest.mark.parametrize("seed", range(60))
def test_tiny_arbitrary_costs(seed):
    """Costs of both signs, negative cycles allowed.

    Theorem on Algorithm 1: an exit with an empty frontier returns V (the
    Kleene limit).  If V has a -inf entry (Kleene diverges) the exit must be
    at the round cap.  The converse does not hold on hypergraphs: a negative
    cycle that the adversary's max can leave through a finite branch has a
    finite value that may need more than |X| rounds; then the cap is hit,
    the iterate stays >= V, and a larger cap reaches V."""
    n = 3 + seed % 5
    K = 1 + seed % 3
    prob = synth.random_small(2000 + seed, n, K)
    r = oracle.solve(prob)
    try:
        kl, _ = brute.kleene(prob)
    except brute.Diverged:
        assert r["status"] == oracle.NEGCYCLE
        return
    V = [math.inf if v == INF_I32 else int(v) for v in r["V"]]
    if r["status"] == oracle.NEGCYCLE:
        assert all(a >= b for a, b in zip(V, kl))
        r = oracle.solve(prob, max_rounds=100 * n)
        V = [math.inf if v == INF_I32 else int(v) for v in r["V"]]
    assert r["status"] == oracle.OK and r["residual"] == 0
    assert V == kl


@pytest.mark.parametrize("seed", range(20))
def test_tiny_float_costs(seed):
    prob = synth.random_small(3000 + seed, 3 + seed % 4, 2, dtype="f32")
    r = oracle.solve(prob, precision="f64")
    try:
        kl, _ = brute.kleene(prob)
    except brute.Diverged:
        assert r["status"] == oracle.NEGCYCLE
        return
    if r["status"] == oracle.NEGCYCLE:
        r = oracle.solve(prob, precision="f64", max_rounds=100 * prob.n)
    assert r["status"] == oracle.OK
    assert r["V"].tolist() == kl


# ---------------------------------------------------------------- Dijkstra
@pytest.mark.parametrize("seed", range(10))
def test_dijkstra_tiny_nonnegative(seed):
    prob = synth.potential_small(4000 + seed, 8 + seed, 3, zero_phi=True)
    assert np.array_equal(oracle.solve(prob)["V"], oracle.dijkstra(prob))


def test_dijkstra_grid2d_nonnegative():
    prob = synth.grid2d_small(phi_top=0.0)
    assert (prob.g >= 1).all()
    r = oracle.solve(prob)
    assert r["status"] == oracle.OK
    assert np.array_equal(r["V"], oracle.dijkstra(prob))


def test_dijkstra_grid4d_nonnegative():
    prob = synth.grid4d(synth.instance_seed(2, 7), dims=(16, 16, 8, 4), phi_top=0.0)
    r = oracle.solve(prob)
    assert r["status"] == oracle.OK
    assert np.array_equal(r["V"], oracle.dijkstra(prob))


# ---------------------------------------------------------------- classical Bellman-Ford
@pytest.mark.parametrize("seed", range(5))
def test_ordinary_digraph_reduces_to_shortest_paths(seed):
    """|F(x,u)| = 1: the problem is a shortest path to a virtual sink with
    edge x -> sink of weight G(x); scipy's Bellman-Ford solves it."""
    from scipy.sparse.csgraph import bellman_ford, csgraph_from_dense
    prob = synth.chain_graph(5000 + seed, 60 + 10 * seed, 3)
    n, K = prob.n, prob.K
    D = np.full((n + 1, n + 1), np.inf)
    for p in range(n * K):
        x, y = p // K, int(prob.succ_idx[prob.succ_ptr[p]])
        D[y, x] = min(D[y, x], float(prob.g[p]))         # reversed edge
    for x in range(n):
        if prob.G[x] < INF_I32:
            D[n, x] = min(D[n, x], float(prob.G[x]))
    dist = bellman_ford(csgraph_from_dense(D, null_value=np.inf), directed=True, indices=n)
    want = np.where(np.isinf(dist[:n]), INF_I32, dist[:n]).astype(np.int64)
    r = oracle.solve(prob)
    assert r["status"] == oracle.OK
    assert np.array_equal(r["V"].astype(np.int64), want)


# ---------------------------------------------------------------- grids
def test_grid2d_vs_kleene():
    prob = synth.grid2d_small()
    r = oracle.solve(prob)
    W, _ = brute.kleene_np(prob)
    assert r["status"] == oracle.OK and r["residual"] == 0
    assert np.array_equal(r["V"], W)


def test_grid2d_float_vs_kleene():
    prob = synth.grid_problem((48, 40), 4, [synth.P_HALF, synth.P_HALF], seed=77, dtype="f32",
                              phi_top=30.0, sigmas=(3, 3, 0, 0), c_range=(0.5, 4.0),
                              target_extent=(4, 4), avoid="iid", avoid_frac=0.1)
    assert (prob.g < 0).any()
    r64 = oracle.solve(prob, precision="f64")
    r32 = oracle.solve(prob, precision="f32")
    assert np.array_equal(r64["V"], brute.kleene_np(prob, np.float64)[0])
    assert np.array_equal(r32["V"], brute.kleene_np(prob, np.float32)[0])
    fin = np.isfinite(r64["V"])
    assert np.array_equal(fin, np.isfinite(r32["V"]))
    scale = np.abs(r64["V"][fin]).max()
    assert np.abs(r64["V"][fin] - r32["V"][fin]).max() <= 1e-5 * scale


def test_grid4d_small_vs_kleene_and_box_decoder():
    prob = synth.grid4d(synth.instance_seed(2, 9), dims=(12, 12, 8, 4))
    ptr, idx = oracle.box_to_csr(prob.dims, prob.box_packed())
    assert np.array_equal(ptr, prob.succ_ptr) and np.array_equal(idx, prob.succ_idx)
    r = oracle.solve(prob)
    assert r["status"] == oracle.OK and r["residual"] == 0
    assert np.array_equal(r["V"], brute.kleene_np(prob)[0])


def _potential_bound_ok(prob, V):
    """For a finite non-target x: V(x) >= phi(x) - max_T phi + c_min, since
    every step costs at least c_min + phi(x) - phi(y) (telescoping)."""
    fin = V < INF_I32 if prob.dtype == "i32" else np.isfinite(V)
    lb = prob.phi.astype(np.float64) - prob.phi[prob.target].max() + prob.c_min
    sel = fin & ~prob.target
    ok_nt = (V[sel].astype(np.float64) >= lb[sel] - 1e-9 * np.abs(lb[sel]).max()).all()
    ok_t = (V[prob.target].astype(np.float64) <= 0).all()
    return ok_nt and ok_t


@pytest.mark.slow
def test_grid4d_full_invariants():
    """4-D 40x40x24x10, 12 inputs, int32: zero residual, the bounds of the
    complexity theorem (rounds <= n, relaxations <= n*m), box decoder, and
    the potential-form lower bound."""
    prob = synth.grid4d()
    r = oracle.solve(prob)
    c = r["counters"]
    assert r["status"] == oracle.OK and r["residual"] == 0
    assert c["rounds"] <= prob.n and c["edge_relax"] <= prob.n * prob.m
    assert _potential_bound_ok(prob, r["V"])
    ptr, idx = oracle.box_to_csr(prob.dims, prob.box_packed())
    assert np.array_equal(ptr, prob.succ_ptr) and np.array_equal(idx, prob.succ_idx)


@pytest.mark.slow
def test_grid4d_fp32_fixed_points():
    """fp32 costs: the double-precision fixed point and the single-precision
    fixed point both have zero residual under their own arithmetic and agree
    to 1e-5 of the value scale."""
    prob = synth.grid4d(dtype="f32")
    r64 = oracle.solve(prob, precision="f64")
    r32 = oracle.solve(prob, precision="f32")
    assert r64["residual"] == 0 and r32["residual"] == 0
    fin = np.isfinite(r64["V"])
    assert np.array_equal(fin, np.isfinite(r32["V"]))
    scale = np.abs(r64["V"][fin]).max()
    assert np.abs(r64["V"][fin] - r32["V"][fin]).max() <= 1e-5 * scale
    assert _potential_bound_ok(prob, r64["V"])
