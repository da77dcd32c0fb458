"""The autotuner on the device: the configuration it picks solves exactly."""
import numpy as np
import pytest

import oracle
import paper_2001_06231_amd as gbf
import synth
from paper_2001_06231_amd import autotune

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    gbf.lib()


def test_tune_single():
    print("\n[case] tune single", flush=True)
    prob = synth.grid4d(synth.instance_seed(60, 0), dims=(12, 10, 6, 4))
    ref = oracle.solve(prob)
    g = gbf.load_problem(prob, encoding="csr")
    opts, ms = gbf.tune([g], reps=2)
    assert opts["mode"] in ("hostloop", "persistent") and opts["lanes"] in (2, 4, 8) and ms > 0
    st, _, V = g.solve(**opts)
    assert st == gbf.OK and np.array_equal(V, ref["V"])
    g.free()


def test_autotune_batch(tmp_path):
    print("\n[case] autotune batch", flush=True)
    import torch
    probs = [synth.grid4d(synth.instance_seed(61, i), dims=(8 + i, 7, 5, 3), K=8) for i in range(4)]
    cache = str(tmp_path / "t.json")
    best = autotune.autotune(probs, reps=2, cache=cache)
    assert best["encoding"] in autotune.ENCODINGS
    graphs = [gbf.load_problem(p, encoding=best["encoding"]) for p in probs]
    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p in probs]
    st, _, _ = gbf.solve_batch(graphs, outs, mode=best["mode"], lanes=best["lanes"], grid=best["grid"])
    assert st == gbf.OK
    for p, v in zip(probs, outs):
        assert np.array_equal(v.cpu().numpy(), oracle.solve(p)["V"])
    for g in graphs:
        g.free()
    assert autotune.autotune(probs, cache=cache) == best


def test_tune_within_a_mode():
    """gbf_tune restricted to one launch mode returns that mode's best
    configuration, which solves exactly; a mode without candidates (one
    workgroup for a batch, persistent with the bucket order) is rejected."""
    print("\n[case] tune within a mode", flush=True)
    import torch
    prob = synth.grid4d(synth.instance_seed(60, 1), dims=(12, 10, 6, 4))
    ref = oracle.solve(prob)
    g = gbf.load_problem(prob, encoding="box+rev")
    for mode in ("hostloop", "persistent", "single_block"):
        opts, ms = gbf.tune([g], reps=1, mode=mode)
        assert opts["mode"] == mode and ms > 0, (mode, opts)
        st, _, V = g.solve(**opts)
        assert st == gbf.OK and np.array_equal(V, ref["V"]), mode
    g2 = gbf.load_problem(synth.grid4d(synth.instance_seed(60, 2), dims=(10, 9, 6, 4)), encoding="box+rev")
    with pytest.raises(gbf.GbfError) as e:
        gbf.tune([g, g2], reps=1, mode="single_block")
    assert e.value.code == gbf.EINVAL
    keys = torch.zeros(prob.n, dtype=torch.int16, device="cuda")
    with pytest.raises(gbf.GbfError) as e:
        gbf.tune([g], reps=1, mode="persistent", order="buckets", bucket_key=keys)
    assert e.value.code == gbf.EINVAL
    g.free()
    g2.free()


def test_relax_block_and_compaction_grid():
    """The host-loop knobs the autotuner searches (relax block size, relax
    grid, compaction grid) change the schedule only: every setting gives the
    oracle's values, in one instance and in a batch; bad values are a clear
    GBF_EINVAL."""
    print("\n[case] relax block and compaction grid", flush=True)
    import torch
    prob = synth.grid4d(synth.instance_seed(60, 3), dims=(14, 11, 6, 4))
    ref = oracle.solve(prob)
    for enc in ("csr", "box+rev"):
        g = gbf.load_problem(prob, encoding=enc)
        for block in (64, 256, 512, 1024):
            for grid, cg in ((0, 0), (8, 1), (4096, 7), (2048, 8192)):
                st, s, V = g.solve(mode="hostloop", block=block, grid=grid, compact_grid=cg)
                assert st == gbf.OK and np.array_equal(V, ref["V"]), (enc, block, grid, cg)
                assert s["block_used"] == block
        for bad in ({"block": 100}, {"block": 2048}, {"block": -64}, {"compact_grid": -1}):
            with pytest.raises(gbf.GbfError) as e:
                g.solve(mode="hostloop", **bad)
            assert e.value.code == gbf.EINVAL, bad
        g.free()
    probs = [synth.grid4d(synth.instance_seed(60, 4 + i), dims=(9 + i, 8, 5, 3), K=8) for i in range(3)]
    graphs = [gbf.load_problem(p, encoding="box+rev") for p in probs]
    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p in probs]
    for block in (128, 1024):
        st, _, _ = gbf.solve_batch(graphs, outs, mode="hostloop", block=block, compact_grid=3)
        assert st == gbf.OK
        for p, v in zip(probs, outs):
            assert np.array_equal(v.cpu().numpy(), oracle.solve(p)["V"]), block
    for gr in graphs:
        gr.free()
