"""Pins of the oracle's sampled fixed-point check (one application of the
operator P of Sect. III-C at chosen states, with the oracle's own box
decoding), which certifies solutions of problems too large for Algorithm 1
on the CPU, and of the paper-scale input generator that feeds it."""
import numpy as np
import pytest

import oracle
import synth
from synth import paper_scale as ps


def _rows(prob, xs):
    K = prob.K
    pid = (xs[:, None] * K + np.arange(K)[None, :]).reshape(-1)
    return prob.box_packed()[pid], np.asarray(prob.g, dtype=np.int32)[pid], np.asarray(prob.G)[xs]


def _sampled(prob, V, xs):
    b, g, G = _rows(prob, xs)
    return oracle.residual_box_sample(prob.dims, prob.K, xs, b, g, G, prob.avoid, V)


@pytest.fixture(scope="module", params=[0, 1, 2])
def solved(request):
    i = request.param
    if i == 0:
        prob = synth.grid2d_small()
    elif i == 1:
        prob = synth.grid4d(synth.instance_seed(2, 21), dims=(12, 10, 6, 4))
    else:
        prob = synth.grid3d(synth.instance_seed(2, 22), dims=(16, 14, 8), K=6)
    return prob, oracle.solve(prob)


def test_fixed_point_passes_at_every_state(solved):
    prob, ref = solved
    xs = np.arange(prob.n, dtype=np.int64)
    bad, _ = _sampled(prob, ref["V"], xs)
    assert bad == 0 and ref["residual"] == 0


def test_counts_equal_the_full_residual_on_perturbed_values(solved):
    """Perturbed value functions: the sampled check over all states counts
    exactly the states that the oracle's full residual (CSR rows from its
    own decoder, the policy pass) counts."""
    prob, ref = solved
    xs = np.arange(prob.n, dtype=np.int64)
    r = synth.Stream(5150, 1)
    fin = np.nonzero((ref["V"] != synth.INF_I32) & (prob.avoid == 0))[0]
    for trial in range(6):
        V = ref["V"].copy()
        pick = fin[r.integers(0, fin.size - 1, 1 + trial * 3)]
        delta = r.integers(-3, 3, pick.size)
        delta[delta == 0] = 1
        V[pick] = V[pick] + delta.astype(np.int32)
        if trial == 5:
            V[fin[0]] = synth.INF_I32  # a finite value replaced by INF
        full, _ = oracle.residual(prob, V)
        bad, first = _sampled(prob, V, xs)
        assert bad == full and bad > 0, (trial, bad, full)


def test_counts_add_over_disjoint_samples(solved):
    prob, ref = solved
    V = ref["V"].copy()
    fin = np.nonzero((V != synth.INF_I32) & (prob.avoid == 0))[0]
    V[fin[::7]] -= 1
    xs = np.arange(prob.n, dtype=np.int64)
    a, b = xs[::2], xs[1::2]
    assert _sampled(prob, V, a)[0] + _sampled(prob, V, b)[0] == _sampled(prob, V, xs)[0] > 0


def test_avoid_state_with_a_finite_value_is_flagged(solved):
    prob, ref = solved
    av = np.nonzero(prob.avoid)[0]
    if av.size == 0:
        pytest.skip("no avoid cells")
    V = ref["V"].copy()
    V[av[0]] = 5
    bad, first = _sampled(prob, V, np.array([av[0]], dtype=np.int64))
    assert bad == 1 and first[0] == av[0]


def test_box_outside_the_grid_is_rejected():
    prob = synth.grid2d_small()
    xs = np.array([0], dtype=np.int64)
    b, g, G = _rows(prob, xs)
    b = b.copy()
    b[0] = np.uint64(prob.n + 5)
    with pytest.raises(ValueError):
        oracle.residual_box_sample(prob.dims, prob.K, xs, b, g, G, prob.avoid, oracle.solve(prob)["V"])


# ---------------------------------------------------------------- generator
@pytest.fixture(scope="module")
def meta():
    return ps.meta()


def test_paper_scale_hash_is_splitmix64(meta):
    import torch
    z = np.arange(4096, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15) + np.uint64(meta["state"])
    a = synth._mix64(z)
    b = ps.mix64_torch(torch.from_numpy(z.view(np.int64))).numpy().view(np.uint64)
    assert np.array_equal(a, b)


def test_paper_scale_rows(meta):
    """Sampled pairs of the 141.75 M-cell grid: boxes lie in the grid and
    follow the drift placement, costs are in potential form (so no negative
    cycle exists), rows do not depend on how the ids are chunked."""
    import torch
    K, dims = ps.K, ps.DIMS
    r = synth.Stream(77, 1)
    pids = np.unique(r.integers(0, meta["n"] * K - 1, 20000)).astype(np.int64)
    box, g = ps.pair_rows(torch.from_numpy(pids), meta)
    box = box.numpy().view(np.uint64)
    g = g.numpy()
    half = pids.size // 2
    b2, g2 = ps.pair_rows(torch.from_numpy(pids[half:]), meta)
    assert np.array_equal(b2.numpy().view(np.uint64), box[half:]) and np.array_equal(g2.numpy(), g[half:])
    ptr, idx = oracle.box_to_csr(dims, box)  # the oracle's decoder: raises if a box leaves the grid
    x = pids // K
    u = pids % K
    st = np.array([1, dims[0], dims[0] * dims[1], dims[0] * dims[1] * dims[2]])
    xc = (x[:, None] // st[None, :]) % np.array(dims)[None, :]
    phi = sum(np.asarray(meta["profiles"][a])[xc[:, a]] for a in range(4))
    for i in range(pids.size):
        ys = idx[ptr[i]:ptr[i + 1]].astype(np.int64)
        yc = (ys[:, None] // st[None, :]) % np.array(dims)[None, :]
        d = meta["drift"][u[i]]
        for a in range(4):
            if d[a] > 0:
                assert yc[:, a].min() >= min(xc[i, a] + d[a], dims[a] - 1)
            elif d[a] < 0:
                assert yc[:, a].max() <= max(xc[i, a] + d[a], 0)
        assert len(ys) <= 16
        phiy = sum(np.asarray(meta["profiles"][a])[yc[:, a]] for a in range(4))
        # g = c + phi(x) - min phi over the box with c >= 1
        assert g[i] >= 1 + phi[i] - phiy.min() and g[i] <= 8 + phi[i] - phiy.min()


def test_paper_scale_target_and_obstacles(meta):
    import torch
    xs = torch.arange(0, meta["n"], 9973, dtype=torch.int64)
    G, av = ps.state_rows(xs, meta)
    G, av = G.numpy(), av.numpy()
    assert not ((G == 0) & (av == 1)).any()
    assert meta["foot"].mean() >= 0.05
    t0, t1 = meta["target"]
    x0 = xs.numpy() % ps.DIMS[0]
    x1 = (xs.numpy() // ps.DIMS[0]) % ps.DIMS[1]
    assert np.array_equal(G == 0, (x0 >= t0) & (x0 < t0 + 6) & (x1 >= t1) & (x1 < t1 + 6))
