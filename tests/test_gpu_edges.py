"""GPU parity of per-edge running costs, g(x,y,u) = g(x,u) + h(x,y,u): values
and canonical policy bit-exact with the oracle for int32 costs and with the
oracle's single-precision operator for fp32 costs (plus the 1e-5 value-scale
check against its double-precision solution), in every solver mode, in the
bucket order and in batches mixed with per-pair-cost instances."""
import copy

import numpy as np
import pytest

import oracle
import paper_2001_06231_amd as gbf
import synth

pytestmark = pytest.mark.gpu

MODES = ["hostloop", "persistent", "single_block"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    gbf.lib()


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _solve(prob, **kw):
    gr = gbf.load_problem(prob)
    status, stats, V = gr.solve(**kw)
    pol, res = gr.policy()
    gr.free()
    return status, stats, V, pol, res


def _exact(ref, got, label):
    status, stats, V, pol, res = got
    assert status == gbf.OK, (label, status)
    assert res == 0, (label, "residual", res)
    bad = np.nonzero(V != ref["V"])[0]
    assert bad.size == 0, (label, "V differs at", bad[:10], V[bad[:10]], ref["V"][bad[:10]])
    badp = np.nonzero(pol != ref["policy"])[0]
    assert badp.size == 0, (label, "policy differs at", badp[:10])


@pytest.fixture(scope="module")
def grid2d_edges():
    prob = synth.with_edge_costs(synth.grid2d_small(), 31)
    return prob, oracle.solve(prob)


@pytest.fixture(scope="module")
def grid4d_edges():
    prob = synth.with_edge_costs(synth.grid4d(synth.instance_seed(2, 21), dims=(14, 13, 8, 4)), 32)
    return prob, oracle.solve(prob)


@pytest.mark.parametrize("seed", range(12))
def test_tiny_edges(seed):
    prob = synth.potential_small_edges(6100 + seed, 5 + seed % 6, 2 + seed % 3)
    _case(f"tiny edges {seed}")
    ref = oracle.solve(prob)
    for mode in MODES:
        _exact(ref, _solve(prob, mode=mode), f"tiny-{seed}-{mode}")


@pytest.mark.parametrize("mode", MODES + ["auto"])
def test_grid2d_edges(grid2d_edges, mode):
    prob, ref = grid2d_edges
    _case(f"grid2d edges {mode}")
    _exact(ref, _solve(prob, mode=mode), f"grid2d-{mode}")


@pytest.mark.parametrize("mode", ["hostloop", "persistent"])
@pytest.mark.parametrize("lanes", [1, 4, 16])
def test_grid4d_edges(grid4d_edges, mode, lanes):
    prob, ref = grid4d_edges
    _case(f"grid4d edges {mode} lanes {lanes}")
    _exact(ref, _solve(prob, mode=mode, lanes=lanes), f"grid4d-{mode}-{lanes}")


def test_grid4d_edges_buckets(grid4d_edges):
    """The bucket order (keys from the oracle's V) leaves the values alone."""
    import torch
    prob, ref = grid4d_edges
    _case("grid4d edges buckets")
    V = ref["V"].astype(np.int64)
    fin = V < oracle.INF_I32
    k = np.zeros(prob.n, np.int64)
    k[fin] = (V[fin] - V[fin].min()) // 8
    keys = torch.from_numpy(np.clip(k, 0, 65535).astype(np.uint16).view(np.int16)).cuda()
    gr = gbf.load_problem(prob)
    status, st, Vb = gr.solve(order="buckets", bucket_key=keys)
    pol, res = gr.policy()
    gr.free()
    _exact(ref, (status, st, Vb, pol, res), "grid4d-buckets")


def test_zero_edge_costs_equal_pair_costs(grid4d_edges):
    """h = 0 everywhere reaches exactly the per-pair problem's result."""
    prob, _ = grid4d_edges
    base = copy.copy(prob)
    base.g_edge = None
    base.g = np.asarray(prob.g)
    z = copy.copy(base)
    z.g_edge = np.zeros(int(prob.succ_ptr[-1]), np.int32)
    _case("zero edge costs")
    a, b = _solve(base), _solve(z)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_grid4d_edges_fp32():
    prob = synth.with_edge_costs(synth.grid4d(synth.instance_seed(2, 22), dtype="f32", dims=(14, 13, 8, 4)), 33,
                                 extra=(0.0, 1.5))
    _case("grid4d edges fp32")
    ref32 = oracle.solve(prob, precision="f32")
    ref64 = oracle.solve(prob, precision="f64")
    for mode in ["hostloop", "persistent"]:
        got = _solve(prob, mode=mode)
        _exact(ref32, got, f"fp32-{mode}")
        V = got[2].astype(np.float64)
        fin = np.isfinite(ref64["V"])
        assert np.array_equal(fin, np.isfinite(V))
        scale = np.abs(ref64["V"][fin]).max()
        assert np.abs(V[fin] - ref64["V"][fin]).max() <= 1e-5 * scale


@pytest.mark.parametrize("mode", ["hostloop", "persistent"])
def test_batch_mixed_with_edge_costs(mode):
    """Per-edge and per-pair instances, CSR and box encodings, in one
    batch: every instance exact."""
    import torch
    s = lambda i: synth.instance_seed(41, i)  # noqa: E731
    items = [
        (synth.with_edge_costs(synth.grid4d(s(0), dims=(10, 9, 6, 4), K=8), 51), "csr"),
        (synth.grid4d(s(1), dims=(12, 10, 6, 4), K=12), "csr"),
        (synth.with_edge_costs(synth.grid2d_small(s(2)), 52), "csr"),
        (synth.grid4d(s(3), dims=(11, 9, 5, 4), K=8), "box+rev"),
        (synth.grid4d(s(4), dims=(8, 8, 4, 3), K=12), "box"),
    ]
    _case(f"batch mixed edges {mode}")
    refs = [oracle.solve(p) for p, _ in items]
    graphs = [gbf.load_problem(p, encoding=e) for p, e in items]
    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p, _ in items]
    status, stats, _ = gbf.solve_batch(graphs, outs, mode=mode)
    assert status == gbf.OK
    for (p, e), gr, V, ref in zip(items, graphs, outs, refs):
        Vh = V.cpu().numpy()
        bad = np.nonzero(Vh != ref["V"])[0]
        assert bad.size == 0, (p.name, e, bad[:8])
        pol, res = gr.policy()
        assert res == 0 and np.array_equal(pol, ref["policy"]), (p.name, e)
    for gr in graphs:
        gr.free()


def test_batch_all_edge_costs():
    import torch
    s = lambda i: synth.instance_seed(42, i)  # noqa: E731
    items = [synth.with_edge_costs(synth.grid4d(s(i), dims=(9 + i, 8, 5, 3), K=8), 60 + i) for i in range(4)]
    _case("batch all edges")
    refs = [oracle.solve(p) for p in items]
    graphs = [gbf.load_problem(p) for p in items]
    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p in items]
    status, stats, _ = gbf.solve_batch(graphs, outs)
    assert status == gbf.OK
    for p, V, ref in zip(items, outs, refs):
        assert np.array_equal(V.cpu().numpy(), ref["V"]), p.name
    for gr in graphs:
        gr.free()


@pytest.mark.timeout(300)
def test_grid4d_384k_edges_full_size():
    """The 4-D 40x40x24x10 graph with per-edge costs, in the launch
    configuration of the benchmark: values and policy exact."""
    prob = synth.with_edge_costs(synth.grid4d(), 34)
    _case("grid4d 384k edges")
    ref = oracle.solve(prob)
    _exact(ref, _solve(prob), "grid4d-384k-edges")


def test_rejects_bad_edge_costs():
    """Non-finite per-edge costs are refused at load; so are per-edge costs
    with the box encoding."""
    prob = synth.potential_small_edges(6200, 6, 2)
    bad = copy.copy(prob)
    bad.g_edge = np.array(prob.g_edge, np.int32)
    bad.g_edge[3] = 2**31 - 1
    with pytest.raises(gbf.GbfError):
        gbf.load_problem(bad)
    pf = synth.potential_small_edges(6201, 6, 2, dtype="f32")
    badf = copy.copy(pf)
    badf.g_edge = np.array(pf.g_edge, np.float32)
    badf.g_edge[1] = np.nan
    with pytest.raises(gbf.GbfError):
        gbf.load_problem(badf)
    with pytest.raises(ValueError):
        gbf.load_problem(prob, encoding="box")


def test_chained_solves():
    """Two problems in sequence, the second terminating in the first's
    value function (G2 = V1, the paper's two-problem mission of Sect. VI-A),
    the second with per-edge costs: exact against the oracle's chain."""
    p1 = synth.grid2d_small()
    _case("chained G2 = V1")
    r1 = oracle.solve(p1)
    st1 = _solve(p1)
    _exact(r1, st1, "chain-1")
    p2 = synth.with_edge_costs(synth.grid2d_small(synth.instance_seed(1, 5)), 36)
    p2.avoid = p1.avoid.copy()
    p2.G = st1[2].astype(np.int32)   # the GPU's V1 (equal to the oracle's)
    r2 = oracle.solve(p2)
    assert r2["status"] == oracle.OK
    _exact(r2, _solve(p2), "chain-2")
    # chaining can only lower values: V2 <= G2 = V1
    assert (r2["V"].astype(np.int64) <= r1["V"].astype(np.int64)).all()


@pytest.mark.parametrize("mode", MODES)
def test_reward_chain(mode):
    """The chained reward workload (synth.reward_problem: G2 = V1 of the
    return problem, per-edge reward for entering the fire region), the
    second problem solved on the GPU with the oracle's V1 as G2: exact
    against the oracle."""
    p1 = synth.grid4d(synth.instance_seed(2, 41), dims=(16, 14, 8, 6))
    r1 = oracle.solve(p1)
    p2 = synth.reward_problem(p1, r1["V"], 101)
    _case(f"reward chain 16x14x8x6 {mode}")
    _exact(oracle.solve(p2), _solve(p2, mode=mode), f"reward-{mode}")


def test_reward_chain_full_size():
    """The same at 40x40x24x10, in the host-loop mode the bench times, with
    G2 = the GPU's own V1 (the chain as the bench runs it; the GPU's V1 is
    checked against the oracle's first)."""
    p1 = synth.grid4d()
    r1 = oracle.solve(p1)
    _case("reward chain 40x40x24x10 hostloop")
    st1 = _solve(p1, mode="hostloop")
    _exact(r1, st1, "reward-full-1")
    p2 = synth.reward_problem(p1, st1[2], 7)
    _exact(oracle.solve(p2), _solve(p2, mode="hostloop"), "reward-full-2")


@pytest.mark.parametrize("seed", range(16))
def test_tiny_edges_arbitrary_sign(seed):
    """Per-edge costs of both signs, negative cycles possible: a diverging
    Kleene iteration must end at the round cap on the GPU; otherwise the
    GPU's values are the Kleene limit."""
    import math
    from oracle import brute
    n, K = 3 + seed % 5, 1 + seed % 3
    prob = synth.random_small_edges(7100 + seed, n, K)
    _case(f"tiny edges arbitrary seed={seed}")
    mode = MODES[seed % 3]
    gr = gbf.load_problem(prob)
    status, stats, V = gr.solve(mode=mode)
    try:
        kl, _ = brute.kleene(prob)
    except brute.Diverged:
        assert status == gbf.ENEGCYCLE
        gr.free()
        return
    if status == gbf.ENEGCYCLE:
        status, stats, V = gr.solve(mode=mode, max_rounds=100 * n)
    assert status == gbf.OK
    assert [math.inf if v == 2**31 - 1 else int(v) for v in V] == kl
    gr.free()
