"""The allocation-free solve (gbf_solve_noalloc) through the C ABI: every
scratch buffer comes from the library's static device array.  Its values
and policy must equal those of gbf_solve on the same handle (bit for bit:
both run the same kernels on the same inputs, and the fixed point does not
depend on processing order), over consecutive calls whose second input is
smaller than the first (the array keeps the last call's contents), and the
calls after the first must not change the device's free memory."""
import numpy as np
import pytest

import paper_2001_06231_amd as gbf
import synth

pytestmark = pytest.mark.gpu

MiB = 1 << 20


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    gbf.lib()


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _reference(gr, n, tdt):
    import torch
    V = torch.empty(n, dtype=tdt, device="cuda")
    status, st, _ = gr.solve(V)
    assert status == gbf.OK
    pol, res = gr.policy()
    assert res == 0
    return V.cpu().numpy(), pol


def _free_bytes():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_noalloc_equals_solve_large_then_small():
    """4-D 40x40x24x10 int32 (4.6 M pairs) then 2-D 64x64 (16 k pairs), then
    the 4-D problem again; each result equals gbf_solve's."""
    import torch
    big = synth.grid4d()
    small = synth.grid2d_small()
    g_big = gbf.load_problem(big, encoding="csr")
    g_small = gbf.load_problem(small, encoding="csr")
    ref_big = _reference(g_big, big.n, torch.int32)
    ref_small = _reference(g_small, small.n, torch.int32)
    frees = []
    for step, (gr, prob, ref) in enumerate([(g_big, big, ref_big), (g_small, small, ref_small),
                                            (g_big, big, ref_big)]):
        _case(f"noalloc call {step}: {prob.name}")
        V = torch.full((prob.n,), -7, dtype=torch.int32, device="cuda")
        before = _free_bytes()
        status, st, _ = gr.solve_noalloc(V)
        after = _free_bytes()
        if step > 0:
            frees.append(before - after)
        assert status == gbf.OK, status
        assert np.array_equal(V.cpu().numpy(), ref[0]), (step, prob.name)
        pol, res = gr.policy()
        assert res == 0 and np.array_equal(pol, ref[1]), (step, prob.name)
        assert st["rounds"] > 0 and st["edge_relax"] > 0
    # the scratch of a 4.6 M-pair solve is ~28 MiB; the calls take none
    assert max(frees) < 2 * MiB, frees
    g_big.free()
    g_small.free()


@pytest.mark.parametrize("mode", ["hostloop", "persistent", "single_block"])
def test_noalloc_modes_fp32_and_host_output(mode):
    """fp32 values (bit patterns) in every solver mode, V written to a host
    array, then a smaller int32 problem."""
    import torch
    prob = synth.grid4d(synth.instance_seed(2, 12), dtype="f32", dims=(12, 10, 6, 4))
    small = synth.grid4d(synth.instance_seed(2, 11), dims=(8, 6, 4, 3), K=8)
    gr = gbf.load_problem(prob, encoding="csr")
    gs = gbf.load_problem(small, encoding="box+rev")
    ref = _reference(gr, prob.n, torch.float32)
    ref_s = _reference(gs, small.n, torch.int32)
    _case(f"noalloc fp32 {mode}")
    status, st, V = gr.solve_noalloc(mode=mode)  # host output
    assert status == gbf.OK
    assert np.array_equal(V.view(np.int32), ref[0].view(np.int32))
    pol, res = gr.policy()
    assert res == 0 and np.array_equal(pol, ref[1])
    _case(f"noalloc smaller int32 {mode}")
    Vs = torch.full((small.n,), -7, dtype=torch.int32, device="cuda")
    status, st, _ = gs.solve_noalloc(Vs, mode=mode)
    assert status == gbf.OK
    assert np.array_equal(Vs.cpu().numpy(), ref_s[0])
    gr.free()
    gs.free()


def test_noalloc_rejects_oversized_problems():
    """More pairs than the static scratch holds, or a larger round cap: a
    clear GBF_EINVAL before any device work; the next call still works."""
    import torch
    n, K = gbf.NOALLOC_MAX_PAIRS // 4 + 1, 4  # one state over the limit
    np_ = n * K
    ptr = np.arange(np_ + 1, dtype=np.int64)
    idx = (np.arange(np_, dtype=np.int64) // K).astype(np.int32)
    g = np.ones(np_, dtype=np.int32)
    G = np.full(n, gbf.INF_I32, dtype=np.int32)
    G[0] = 0
    _case("noalloc over the pair limit")
    gr = gbf.load_graph(n, K, G, g, succ_ptr=ptr, succ_idx=idx)
    with pytest.raises(gbf.GbfError) as e:
        gr.solve_noalloc()
    assert e.value.code == gbf.EINVAL and "pairs" in str(e.value)
    gr.free()
    small = synth.grid2d_small()
    gs = gbf.load_problem(small)
    _case("noalloc over the round-cap limit")
    with pytest.raises(gbf.GbfError) as e:
        gs.solve_noalloc(max_rounds=gbf.NOALLOC_MAX_ROUNDS + 1)
    assert e.value.code == gbf.EINVAL
    import ctypes
    L = gbf.lib()
    o = gbf._Opts()
    o.order = gbf.ORDER_BUCKETS
    o.v_memspace = gbf.HOST
    out = np.empty(small.n, dtype=np.int32)
    assert L.gbf_solve_noalloc(gs._h, ctypes.byref(o), out.ctypes.data, None) == gbf.EINVAL
    ref = _reference(gs, small.n, torch.int32)
    status, st, V = gs.solve_noalloc()
    assert status == gbf.OK and np.array_equal(V, ref[0])
    gs.free()
