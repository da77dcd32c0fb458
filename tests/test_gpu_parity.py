"""GPU parity: the HIP path through the C ABI against the CPU oracle.

int32 costs: values and canonical policy bit-exact.  fp32 costs: values
bit-exact with the oracle's single-precision operator (one IEEE RNE addition
per backup, whose maximal fixed point is unique and order-independent), and
within 1e-5 relative of the oracle's double-precision solution element by
element (|V| floored at one cost unit), with an identical policy wherever
the value gap exceeds that tolerance.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2001_06231_amd as gbf
import synth
from oracle import brute
from tests import golden_io

pytestmark = pytest.mark.gpu

INF_I32 = 2**31 - 1
MODES = ["hostloop", "persistent"]
SMALL_MODES = MODES + ["single_block"]  # the one-workgroup solver, for small instances


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    gbf.lib()


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _gpu_solve(prob, encoding="csr", mode="auto", **kw):
    gr = gbf.load_problem(prob, encoding=encoding)
    status, stats, V = gr.solve(mode=mode, **kw)
    pol, res = gr.policy()
    gr.free()
    return status, stats, V, pol, res


def _assert_exact(prob, ref, got, label):
    status, stats, V, pol, res = got
    assert status == gbf.OK, (label, status)
    assert res == 0, (label, "residual", res)
    bad = np.nonzero(V != ref["V"])[0]
    assert bad.size == 0, (label, "V differs at", bad[:10], V[bad[:10]], ref["V"][bad[:10]])
    badp = np.nonzero(pol != ref["policy"])[0]
    assert badp.size == 0, (label, "policy differs at", badp[:10], pol[badp[:10]], ref["policy"][badp[:10]])


# ------------------------------------------------------------------ worked example
@pytest.mark.parametrize("mode", SMALL_MODES)
def test_fig2_example(mode):
    prob, inputs, facts = golden_io.load("fig2_example.txt")
    _case(f"fig2 {mode}")
    ref = oracle.solve(prob)
    _assert_exact(prob, ref, _gpu_solve(prob, mode=mode), "fig2")


@pytest.mark.parametrize("mode", SMALL_MODES)
def test_negative_cycle_status(mode):
    prob, _, _ = golden_io.load("negcycle.txt")
    _case(f"negcycle {mode}")
    gr = gbf.load_problem(prob)
    status, stats, V = gr.solve(mode=mode)
    assert status == gbf.ENEGCYCLE
    assert stats["rounds"] == prob.n
    gr.free()


# ------------------------------------------------------------------ tiny brute force
@pytest.mark.parametrize("seed", range(24))
def test_tiny_potential_form(seed):
    n, K = 3 + seed % 6, 1 + seed % 3
    prob = synth.potential_small(6000 + seed, n, K)
    _case(f"tiny potential seed={seed} n={n} K={K}")
    ref = oracle.solve(prob)
    _assert_exact(prob, ref, _gpu_solve(prob, mode=SMALL_MODES[seed % 3]), f"tiny{seed}")


@pytest.mark.parametrize("seed", range(24))
def test_tiny_arbitrary_costs(seed):
    """Both signs, negative cycles possible: if V has -inf (Kleene diverges)
    the GPU must stop at the cap; if the GPU's frontier drains its V must be
    the Kleene limit."""
    n, K = 3 + seed % 5, 1 + seed % 3
    prob = synth.random_small(7000 + seed, n, K)
    _case(f"tiny arbitrary seed={seed} n={n} K={K}")
    gr = gbf.load_problem(prob)
    status, stats, V = gr.solve(mode=SMALL_MODES[seed % 3])
    try:
        kl, _ = brute.kleene(prob)
    except brute.Diverged:
        assert status == gbf.ENEGCYCLE
        return
    if status == gbf.ENEGCYCLE:
        status, stats, V = gr.solve(mode=SMALL_MODES[seed % 3], max_rounds=100 * n)
    assert status == gbf.OK
    assert [math.inf if v == INF_I32 else int(v) for v in V] == kl
    gr.free()


# ------------------------------------------------------------------ grids
@pytest.fixture(scope="module")
def grid2d():
    prob = synth.grid2d_small()
    return prob, oracle.solve(prob)


@pytest.mark.parametrize("encoding", ["csr", "box", "box+rev"])
@pytest.mark.parametrize("mode", SMALL_MODES)
def test_grid2d_64x64(grid2d, encoding, mode):
    prob, ref = grid2d
    _case(f"grid2d 64x64 {encoding} {mode}")
    _assert_exact(prob, ref, _gpu_solve(prob, encoding, mode), f"grid2d-{encoding}-{mode}")


@pytest.mark.parametrize("grid,lanes", [(1, 1), (3, 2), (64, 4), (2048, 8), (4096, 16), (512, 32)])
def test_grid2d_launch_shapes(grid2d, grid, lanes):
    """Results do not depend on the number of blocks or lanes per pair (a
    race would show as a launch-shape dependence)."""
    prob, ref = grid2d
    _case(f"grid2d grid={grid} lanes={lanes}")
    for enc in ("csr", "box", "box+rev"):
        _assert_exact(prob, ref, _gpu_solve(prob, enc, "hostloop", grid=grid, lanes=lanes), f"grid{grid}")
        _assert_exact(prob, ref, _gpu_solve(prob, enc, "persistent", grid=grid, lanes=lanes), f"pgrid{grid}")


@pytest.mark.parametrize("encoding", ["csr", "box", "box+rev"])
@pytest.mark.parametrize("mode", ["persistent", "single_block"])
def test_grid4d_small(encoding, mode):
    prob = synth.grid4d(synth.instance_seed(2, 11), dims=(14, 12, 8, 5))
    _case(f"grid4d 14x12x8x5 {encoding} {mode}")
    ref = oracle.solve(prob)
    _assert_exact(prob, ref, _gpu_solve(prob, encoding, mode), "grid4d-small")


@pytest.mark.parametrize("lanes", [1, 4, 32])
def test_single_block_fp32_and_lanes(lanes):
    prob = synth.grid4d(synth.instance_seed(2, 12), dtype="f32", dims=(12, 10, 6, 4))
    _case(f"single block fp32 lanes={lanes}")
    ref = oracle.solve(prob, precision="f32")
    _assert_exact(prob, ref, _gpu_solve(prob, "csr", "single_block", lanes=lanes), "single-fp32")


@pytest.fixture(scope="module")
def grid4d_full():
    prob = synth.grid4d()
    return prob, oracle.solve(prob)


@pytest.mark.parametrize("encoding", ["csr", "box", "box+rev"])
@pytest.mark.parametrize("mode", MODES)
def test_grid4d_40x40x24x10_int32(grid4d_full, encoding, mode):
    prob, ref = grid4d_full
    _case(f"grid4d 40x40x24x10 int32 {encoding} {mode}")
    _assert_exact(prob, ref, _gpu_solve(prob, encoding, mode), f"grid4d-{encoding}-{mode}")


@pytest.mark.parametrize("lanes", [1, 2, 8, 32])
def test_grid4d_40x40x24x10_lanes(grid4d_full, lanes):
    prob, ref = grid4d_full
    _case(f"grid4d 40x40x24x10 int32 csr lanes={lanes}")
    _assert_exact(prob, ref, _gpu_solve(prob, "csr", "hostloop", lanes=lanes, grid=4096), f"lanes{lanes}")


@pytest.fixture(scope="module")
def grid4d_f32():
    prob = synth.grid4d(dtype="f32")
    return prob, oracle.solve(prob, precision="f32"), oracle.solve(prob, precision="f64")


@pytest.mark.parametrize("encoding", ["csr", "box", "box+rev"])
@pytest.mark.parametrize("mode", ["auto", "hostloop", "persistent"])
def test_grid4d_40x40x24x10_fp32(grid4d_f32, encoding, mode):
    prob, ref32, ref64 = grid4d_f32
    _case(f"grid4d 40x40x24x10 fp32 {encoding} {mode}")
    got = _gpu_solve(prob, encoding, mode)
    # bit-exact with the single-precision operator
    _assert_exact(prob, ref32, got, f"fp32-{encoding}-{mode}")
    # within 1e-5 relative of the double-precision solution, element by
    # element; values below one cost unit are compared with an absolute
    # 1e-5 (their error is that of the larger partial sums along the path)
    V = got[2].astype(np.float64)
    fin = np.isfinite(ref64["V"])
    assert np.array_equal(fin, np.isfinite(V))
    gap = np.abs(V[fin] - ref64["V"][fin])
    rel = gap / np.maximum(np.abs(ref64["V"][fin]), 1.0)
    assert rel.max() <= 1e-5, rel.max()
    tol_of = lambda v: 1e-5 * max(abs(v), 1.0)  # noqa: E731
    # same controller wherever the fp64 optimum is separated by more than
    # the tolerance: where the policies differ, both choices must have fp64
    # backup values within the tolerance of each other
    pol = got[3]
    differ = np.nonzero(pol != ref64["policy"])[0]
    if differ.size:
        d64 = _backups_f64(prob, ref64["V"])
        for x in differ:
            a = _choice_value(prob, d64, x, int(pol[x]))
            b = _choice_value(prob, d64, x, int(ref64["policy"][x]))
            assert abs(a - b) <= tol_of(b), (x, pol[x], ref64["policy"][x], a, b)


def _backups_f64(prob, V64):
    W = np.where(np.isfinite(V64), V64, np.inf)
    mx = np.maximum.reduceat(W[prob.succ_idx], prob.succ_ptr[:-1].astype(np.intp))
    return prob.g.astype(np.float64) + mx


def _choice_value(prob, d64, x, u):
    if u == gbf.HANDOVER:
        return float(prob.G[x])
    if u == gbf.NONE:
        return math.inf
    return float(d64[x * prob.K + u])
