"""GPU parity of the solver with 64-bit pair ids (the form that problems of
2^31 pairs or more take, e.g. the 141.7 M-state, 35-input problems of
Sect. VI-A).  Here the 64-bit instantiation is forced on problems the
oracle solves in seconds: values and canonical policy must be bit-exact
with the oracle in the implicit box encoding and with the 64-bit reverse
CSR (box successors, relative predecessor entries)."""
import numpy as np
import pytest

import oracle
import paper_2001_06231_amd as gbf
import synth

pytestmark = pytest.mark.gpu

ENCODINGS = ["box", "box+rev"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    gbf.lib()


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _solve_wide(prob, encoding, **kw):
    gr = gbf.load_problem(prob, encoding=encoding, pair_ids64=True)
    status, st, V = gr.solve(**kw)
    pol, res = gr.policy()
    gr.free()
    return status, st, V, pol, res


def _exact(label, got, ref):
    status, st, V, pol, res = got
    assert status == gbf.OK, (label, status)
    assert res == 0, (label, "residual", res)
    bad = np.nonzero(V != ref["V"])[0]
    assert bad.size == 0, (label, bad[:8], V[bad[:8]], ref["V"][bad[:8]])
    assert np.array_equal(pol, ref["policy"]), label


@pytest.mark.parametrize("encoding", ENCODINGS)
@pytest.mark.parametrize("lanes", [2, 4, 8])
def test_wide_grid2d(encoding, lanes):
    prob = synth.grid2d_small()
    ref = oracle.solve(prob)
    _case(f"64-bit ids grid2d {encoding} lanes={lanes}")
    _exact(f"grid2d-{encoding}-{lanes}", _solve_wide(prob, encoding, lanes=lanes), ref)


@pytest.mark.parametrize("encoding", ENCODINGS)
def test_wide_grid4d_small_int32_and_fp32(encoding):
    prob = synth.grid4d(synth.instance_seed(2, 11), dims=(14, 12, 8, 5))
    _case(f"64-bit ids grid4d 14x12x8x5 {encoding}")
    _exact(f"grid4d-{encoding}", _solve_wide(prob, encoding), oracle.solve(prob))
    pf = synth.grid4d(synth.instance_seed(2, 12), dtype="f32", dims=(12, 10, 6, 4))
    _case(f"64-bit ids grid4d fp32 {encoding}")
    _exact(f"grid4d-f32-{encoding}", _solve_wide(pf, encoding), oracle.solve(pf, precision="f32"))


@pytest.mark.parametrize("grid", [1, 7, 512, 4096])
def test_wide_launch_shapes(grid):
    """Results do not depend on the relax grid (ragged last waves)."""
    prob = synth.grid4d(synth.instance_seed(2, 13), dims=(11, 9, 6, 4), K=8)
    ref = oracle.solve(prob)
    _case(f"64-bit ids launch grid={grid}")
    for enc in ENCODINGS:
        _exact(f"grid{grid}-{enc}", _solve_wide(prob, enc, grid=grid), ref)


@pytest.fixture(scope="module")
def grid4d_full():
    prob = synth.grid4d()
    return prob, oracle.solve(prob)


@pytest.mark.parametrize("encoding", ENCODINGS)
def test_wide_grid4d_40x40x24x10(grid4d_full, encoding):
    prob, ref = grid4d_full
    _case(f"64-bit ids grid4d 40x40x24x10 {encoding}")
    got = _solve_wide(prob, encoding)
    _exact(f"full-{encoding}", got, ref)
    # the same solve with 32-bit ids evaluates the same kind of work
    assert got[1]["rounds"] > 0 and got[1]["edge_relax"] > 0


def test_wide_memory_budget_choice():
    """expand_box 3 with 64-bit ids: the reverse CSR is built if it fits the
    budget, else the problem stays implicit; exact either way."""
    prob = synth.grid4d(synth.instance_seed(2, 14), dims=(12, 10, 6, 4))
    ref = oracle.solve(prob)
    _case("64-bit ids memory budget")
    for budget, want in ((1 << 40, 2), (1 << 20, 1)):
        gr = gbf.load_problem(prob, encoding="box:budget", mem_budget=budget, pair_ids64=True)
        status, st, V = gr.solve()
        pol, res = gr.policy()
        assert st["enc_used"] == want, (budget, st["enc_used"])
        _exact(f"budget-{budget}", (status, st, V, pol, res), ref)
        gr.free()


def test_wide_rejected_uses():
    """64-bit ids run one instance, in host-loop mode and plain order, from
    boxes; everything else is a clear GBF_EINVAL."""
    import torch
    prob = synth.grid4d(synth.instance_seed(2, 15), dims=(8, 6, 4, 3), K=8)
    _case("64-bit ids rejected uses")
    with pytest.raises(gbf.GbfError) as e:
        gbf.load_graph(prob.n, prob.K, prob.G, prob.g, encoding="csr", avoid=prob.avoid,
                       succ_ptr=prob.ensure_csr().succ_ptr, succ_idx=prob.succ_idx, pair_ids64=True)
    assert e.value.code == gbf.EINVAL
    with pytest.raises(gbf.GbfError) as e:
        gbf.load_problem(prob, encoding="box->csr", pair_ids64=True)
    assert e.value.code == gbf.EINVAL
    gr = gbf.load_problem(prob, encoding="box+rev", pair_ids64=True)
    for kw in ({"mode": "persistent"}, {"mode": "single_block"}):
        with pytest.raises(gbf.GbfError) as e:
            gr.solve(**kw)
        assert e.value.code == gbf.EINVAL, kw
    kt = torch.zeros(prob.n, dtype=torch.int16, device="cuda")
    with pytest.raises(gbf.GbfError) as e:
        gr.solve(order="buckets", bucket_key=kt)
    assert e.value.code == gbf.EINVAL
    with pytest.raises(gbf.GbfError) as e:
        gr.solve_noalloc()
    assert e.value.code == gbf.EINVAL
    g2 = gbf.load_problem(prob, encoding="box", pair_ids64=True)
    with pytest.raises(gbf.GbfError) as e:
        gbf.solve_batch([gr, g2])
    assert e.value.code == gbf.EINVAL
    # the handle still solves
    status, st, V = gr.solve()
    assert status == gbf.OK and np.array_equal(V, oracle.solve(prob)["V"])
    gr.free()
    g2.free()
