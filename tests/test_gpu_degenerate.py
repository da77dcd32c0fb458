"""Degenerate and edge-case inputs through the C ABI against the oracle:
one state, self-loops, no target, every state a target, all cells avoided,
forbidden inputs, chains, more inputs than a wave has lanes (the wide
policy kernel), ragged pair counts, and the 2^31 successor limit."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2001_06231_amd as gbf
import synth

pytestmark = pytest.mark.gpu

INF = 2**31 - 1
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


def _check(prob, mode):
    ref = oracle.solve(prob)
    gr = gbf.load_problem(prob)
    status, st, V = gr.solve(mode=mode)
    want = gbf.OK if ref["status"] == oracle.OK else gbf.ENEGCYCLE
    assert status == want, (status, ref["status"])
    if status == gbf.OK:
        pol, res = gr.policy()
        assert res == 0
        assert np.array_equal(V, ref["V"]) and np.array_equal(pol, ref["policy"])
    gr.free()
    return st, ref


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("g,G", [(2, 5), (0, 5), (-1, 5), (3, INF)])
def test_single_state_self_loop(mode, g, G):
    """One state, one input, F(0,0) = {0}: V = G unless the loop is negative
    (then the round cap ends the solve)."""
    _case(f"one state g={g} G={G} {mode}")
    prob = synth.explicit_problem(1, 1, [[0]], [g], [G])
    st, ref = _check(prob, mode)
    if g >= 0:
        assert int(ref["V"][0]) == G


@pytest.mark.parametrize("mode", MODES)
def test_no_target(mode):
    """G = INF everywhere: nothing is controllable, the frontier starts
    empty, every policy entry is 'none'."""
    _case(f"no target {mode}")
    prob = synth.potential_small(8100, 12, 3)
    prob.G = np.full(prob.n, INF, np.int32)
    st, ref = _check(prob, mode)
    assert (ref["V"] == INF).all() and (ref["policy"] == oracle.NONE).all()
    assert st["rounds"] == 0 and st["pair_evals"] == 0


@pytest.mark.parametrize("mode", MODES)
def test_every_state_a_target(mode):
    _case(f"all targets {mode}")
    prob = synth.potential_small(8101, 15, 2)
    prob.G = np.arange(prob.n, dtype=np.int32) % 7
    _check(prob, mode)


@pytest.mark.parametrize("mode", MODES)
def test_all_cells_avoided(mode):
    _case(f"all avoid {mode}")
    prob = synth.potential_small(8102, 10, 2)
    prob.G = np.full(prob.n, INF, np.int32)
    prob.avoid = np.ones(prob.n, np.uint8)
    st, ref = _check(prob, mode)
    assert (ref["V"] == INF).all()


@pytest.mark.parametrize("mode", MODES)
def test_forbidden_inputs(mode):
    """Some states have every input forbidden (g = INF): they keep G (hand
    over) or INF (none)."""
    _case(f"forbidden inputs {mode}")
    prob = synth.potential_small(8103, 14, 3)
    g = np.array(prob.g, np.int64)
    for x in (0, 3, 7):
        g[x * 3:(x + 1) * 3] = INF
    prob.g = g.astype(np.int32)
    _check(prob, mode)


@pytest.mark.parametrize("mode", MODES)
def test_chain(mode):
    """K = 1 path 0 <- 1 <- ... <- n-1 with unit costs: V(x) = x, n - 1
    rounds of one state each."""
    n = 97
    _case(f"chain {mode}")
    rows = [[max(x - 1, 0)] for x in range(n)]
    G = [0] + [INF] * (n - 1)
    prob = synth.explicit_problem(n, 1, rows, [1] * n, G)
    st, ref = _check(prob, mode)
    assert list(ref["V"]) == list(range(n))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("K", [63, 64, 65, 130])
def test_many_inputs(mode, K):
    """K around and above the wave width (the policy kernel switches to its
    one-state-per-thread form above 64)."""
    _case(f"K={K} {mode}")
    prob = synth.potential_small(8200 + K, 9, K, max_succ=4)
    _check(prob, mode)


@pytest.mark.parametrize("n,K", [(17, 3), (33, 5), (257, 7), (1001, 13)])
def test_ragged_pair_counts(n, K):
    """Pair counts that are not multiples of the 16-pair map chunks."""
    _case(f"ragged n={n} K={K}")
    prob = synth.potential_small(8300 + n, n, K, max_succ=5)
    for mode in MODES:
        _check(prob, mode)


def test_successor_limit_rejected():
    """A successor list total of 2^31 entries is refused before any
    allocation of that size."""
    _case("m >= 2^31")
    n, K = 4, 1
    p = gbf._Problem()
    p.n_states, p.n_inputs, p.dtype, p.encoding, p.memspace = n, K, gbf.I32, gbf.CSR, gbf.HOST
    G = (ctypes.c_int32 * n)(0, 1, 1, 1)
    g = (ctypes.c_int32 * n)(1, 1, 1, 1)
    sp = (ctypes.c_int64 * (n * K + 1))(0, 1, 2, 3, 2**31)
    si = (ctypes.c_int32 * 4)(0, 0, 0, 0)
    p.G, p.g = ctypes.cast(G, ctypes.c_void_p), ctypes.cast(g, ctypes.c_void_p)
    p.succ_ptr, p.succ_idx = ctypes.cast(sp, ctypes.c_void_p), ctypes.cast(si, ctypes.c_void_p)
    h = ctypes.c_void_p()
    L = gbf.lib()
    assert L.gbf_load_graph(ctypes.byref(p), None, ctypes.byref(h)) == gbf.EINVAL
    assert b"2^31" in L.gbf_last_error()


def _check_f32(prob, mode):
    ref = oracle.solve(prob, precision="f32")
    gr = gbf.load_problem(prob)
    status, st, V = gr.solve(mode=mode)
    assert status == gbf.OK and ref["status"] == oracle.OK
    pol, res = gr.policy()
    assert res == 0
    same = (V == ref["V"]) | (np.isnan(V) & np.isnan(ref["V"]))
    assert same.all() and np.array_equal(pol, ref["policy"])
    gr.free()
    return ref


@pytest.mark.parametrize("mode", MODES)
def test_fp32_overflow_and_signed_zero(mode):
    """fp32 sums that overflow to +inf count as INF (no candidate), and
    -0.0 costs and terminal values compare equal to +0.0."""
    _case(f"fp32 overflow / -0 {mode}")
    big = np.float32(3.0e38)
    rows = [[1], [2], [2], [2], [3], [0, 4]]
    g = [big, big, 0.0, -0.0, 1.5, 2.0]     # 0 -> 1 -> 2 costs big + big: overflow
    G = [np.inf, np.inf, -0.0, np.inf, np.inf, np.inf]
    prob = synth.explicit_problem(6, 1, rows, g, G, dtype="f32")
    ref = _check_f32(prob, mode)
    assert ref["V"][1] == big and np.isinf(ref["V"][0])   # big + big overflows
    assert ref["V"][2] == 0.0 and ref["V"][3] == 0.0 and ref["V"][4] == 1.5
    assert np.isinf(ref["V"][5])                          # max over {INF, 1.5}
