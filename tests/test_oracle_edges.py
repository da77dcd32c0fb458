"""Pins of the oracle's per-edge running costs, g(x,y,u) = g(x,u) + h(x,y,u)
(the general running cost of Sect. III-B and the operator of Sect. III-C),
to facts other than itself: the paper's worked example (Fig. 2) restated
with its costs on the edges, brute force from the definitions, the
independent min-max Dijkstra, scipy's Bellman-Ford on ordinary digraphs, and
reductions to per-pair costs."""
import copy
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import brute
from tests import golden_io

INF_I32 = 2**31 - 1


def _as_edges(prob, keep=0):
    """The same problem with each pair's cost moved onto its edges (h = g - keep
    on every entry of the row, g(x,u) = keep)."""
    q = copy.copy(prob)
    rows = np.diff(np.asarray(prob.succ_ptr))
    g = np.asarray(prob.g, dtype=np.int64)
    fin = g < INF_I32
    q.g_edge = np.repeat(np.where(fin, g - keep, 0), rows).astype(np.int32)
    q.g = np.where(fin, keep, INF_I32).astype(np.int32)
    return q


def _v(r):
    return [math.inf if v == INF_I32 else int(v) for v in r["V"]]


def test_fig2_with_edge_costs():
    """Fig. 2 labels its edges with costs (equal within each pair): put them
    on the edges and the paper's value function and controller come out."""
    prob, inputs, facts = golden_io.load("fig2_example.txt")
    want = oracle.solve(prob)
    for keep in (0, 1):
        r = oracle.solve(_as_edges(prob, keep))
        assert r["status"] == oracle.OK and r["residual"] == 0
        assert np.array_equal(r["V"], want["V"])
        names = {int(s) - 1: name for s, name in facts["mu"]}
        for x, name in names.items():
            p = int(r["policy"][x])
            got = "U" if p == oracle.HANDOVER else ("none" if p == oracle.NONE else inputs[p])
            assert got == name


@pytest.mark.parametrize("seed", range(30))
def test_tiny_edges_vs_brute_force(seed):
    n = 3 + seed % 4
    K = 2 + seed % 2
    prob = synth.potential_small_edges(6000 + seed, n, K)
    r = oracle.solve(prob)
    assert r["status"] == oracle.OK and r["residual"] == 0
    V = _v(r)
    assert V == brute.kleene(prob)[0]
    if K ** n <= 4096:
        assert V == brute.enumerate_V(prob)
    L = brute.evaluate(prob, r["policy"].tolist())
    assert [math.inf if v == INF_I32 else v for v in L] == V


@pytest.mark.parametrize("seed", range(40))
def test_tiny_edges_arbitrary_sign(seed):
    """Edge costs of both signs (negative cycles possible): an exit with an
    empty frontier returns the Kleene limit; divergence means the round cap."""
    n = 3 + seed % 5
    K = 1 + seed % 3
    prob = synth.random_small_edges(7000 + seed, n, K)
    r = oracle.solve(prob)
    try:
        kl, _ = brute.kleene(prob)
    except brute.Diverged:
        assert r["status"] == oracle.NEGCYCLE
        return
    if r["status"] == oracle.NEGCYCLE:
        assert all(a >= b for a, b in zip(_v(r), kl))
        r = oracle.solve(prob, max_rounds=100 * n)
    assert r["status"] == oracle.OK and r["residual"] == 0
    assert _v(r) == kl


@pytest.mark.parametrize("seed", range(10))
def test_tiny_edges_float(seed):
    prob = synth.random_small_edges(8000 + seed, 3 + seed % 4, 2, dtype="f32")
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


@pytest.mark.parametrize("seed", range(8))
def test_edges_dijkstra_nonnegative(seed):
    prob = synth.potential_small_edges(9000 + seed, 8 + seed, 3, zero_phi=True)
    assert (prob.g_edge >= 0).all()
    assert np.array_equal(oracle.solve(prob)["V"], oracle.dijkstra(prob))


def test_edges_dijkstra_grid():
    prob = synth.with_edge_costs(synth.grid4d(synth.instance_seed(2, 9), dims=(12, 12, 6, 4), phi_top=0.0), 5)
    assert (prob.g_edge >= 0).all()
    r = oracle.solve(prob)
    assert r["status"] == oracle.OK and r["residual"] == 0
    assert np.array_equal(r["V"], oracle.dijkstra(prob))


@pytest.mark.parametrize("seed", range(4))
def test_ordinary_digraph_edge_costs_shortest_paths(seed):
    """|F(x,u)| = 1 with the whole cost on the edge: shortest paths to a
    virtual sink (scipy's Bellman-Ford)."""
    from scipy.sparse.csgraph import bellman_ford, csgraph_from_dense
    base = synth.chain_graph(5100 + seed, 50 + 10 * seed, 3)
    prob = _as_edges(base)
    n, K = prob.n, prob.K
    D = np.full((n + 1, n + 1), np.inf)
    for p in range(n * K):
        e = int(prob.succ_ptr[p])
        x, y = p // K, int(prob.succ_idx[e])
        D[y, x] = min(D[y, x], float(prob.g_edge[e]))
    for x in range(n):
        if prob.G[x] < INF_I32:
            D[n, x] = min(D[n, x], float(prob.G[x]))
    dist = bellman_ford(csgraph_from_dense(D, null_value=np.inf), directed=True, indices=n)
    want = np.where(np.isinf(dist[:n]), INF_I32, dist[:n]).astype(np.int64)
    r = oracle.solve(prob)
    assert r["status"] == oracle.OK
    assert np.array_equal(r["V"].astype(np.int64), want)


def test_edges_reduce_to_pair_costs():
    """h = 0, or h constant along each row with g lowered by the same
    amount, gives exactly the per-pair problem."""
    prob = synth.grid2d_small()
    want = oracle.solve(prob)
    q = copy.copy(prob)
    q.g_edge = np.zeros(int(prob.succ_ptr[-1]), np.int32)
    r = oracle.solve(q)
    assert np.array_equal(r["V"], want["V"]) and np.array_equal(r["policy"], want["policy"])
    r = oracle.solve(_as_edges(prob, keep=3))
    assert np.array_equal(r["V"], want["V"]) and np.array_equal(r["policy"], want["policy"])


def test_edges_matter():
    """Per-edge costs change the result where the row's max moves: the
    same system with each row's costs replaced by their max differs."""
    prob = synth.with_edge_costs(synth.grid2d_small(), 3)
    r = oracle.solve(prob)
    assert r["status"] == oracle.OK and r["residual"] == 0
    q = copy.copy(prob)
    rows = np.diff(np.asarray(prob.succ_ptr))
    starts = np.asarray(prob.succ_ptr[:-1])
    rowmax = np.maximum.reduceat(prob.g_edge.astype(np.int64), starts)
    q.g_edge = np.repeat(rowmax, rows).astype(np.int32)
    rq = oracle.solve(q)
    assert (rq["V"] >= r["V"]).all() and (rq["V"] > r["V"]).any()


@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_edges_grid_vs_kleene(dtype):
    prob = synth.with_edge_costs(synth.grid4d(synth.instance_seed(2, 11), dtype=dtype, dims=(10, 10, 6, 4)), 9,
                                 extra=(0, 4) if dtype == "i32" else (0.0, 1.5))
    if dtype == "i32":
        r = oracle.solve(prob)
        kl, _ = brute.kleene_np(prob)
        assert r["status"] == oracle.OK and r["residual"] == 0
        assert np.array_equal(r["V"], kl)
    else:
        r = oracle.solve(prob, precision="f32")
        kl, _ = brute.kleene_np(prob, dtype=np.float32)
        assert r["status"] == oracle.OK and r["residual"] == 0
        assert np.array_equal(r["V"], kl)
        r64 = oracle.solve(prob, precision="f64")
        k64, _ = brute.kleene_np(prob, dtype=np.float64)
        assert np.array_equal(r64["V"], k64)
        fin = np.isfinite(k64)
        assert np.array_equal(fin, np.isfinite(r["V"]))
        # single precision stays within 1e-5 of the value range of the double one
        scale = np.abs(k64[fin]).max()
        assert np.abs(r["V"][fin] - k64[fin]).max() <= 1e-5 * scale
