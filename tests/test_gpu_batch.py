"""GPU parity of the batched solver: one frontier over many instances of
uneven size must give, for every instance, exactly what the oracle (and the
single-instance solver) gives."""
import numpy as np
import pytest

import oracle
import paper_2001_06231_amd as gbf
import synth
from tests import golden_io

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    gbf.lib()


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _small_mix(dtype="i32"):
    """Small instances of every family, with their encodings."""
    out = []
    s = lambda i: synth.instance_seed(40, i)  # noqa: E731
    out.append((synth.grid_problem((24, 20), 4, [synth.P_HALF, synth.P_HALF], seed=s(0), dtype=dtype,
                                   phi_top=40.0 if dtype == "i32" else 30.0, sigmas=(3, 3, 0, 0),
                                   c_range=(1, 8) if dtype == "i32" else (0.5, 4.0), target_extent=(4, 4),
                                   avoid="iid", avoid_frac=0.1), "csr"))
    out.append((synth.grid3d(s(1), dims=(12, 10, 6), K=6) if dtype == "i32" else
                synth.grid4d(s(1), dtype=dtype, dims=(9, 8, 5, 3), K=8), "box"))
    out.append((synth.grid4d(s(2), dtype=dtype, dims=(10, 9, 6, 4), K=8), "box->csr"))
    out.append((synth.grid4d(s(3), dtype=dtype, dims=(12, 10, 6, 4), K=12), "csr"))
    out.append((synth.grid4d(s(4), dtype=dtype, dims=(8, 8, 4, 3), K=12), "box"))
    out.append((synth.grid4d(s(5), dtype=dtype, dims=(11, 9, 5, 4), K=8), "box+rev"))
    return out


def _check_batch(items, mode, precision=None, reps=1):
    import torch
    refs = [oracle.solve(p, precision=precision) for p, _ in items]
    graphs = [gbf.load_problem(p, encoding=e) for p, e in items]
    tdt = torch.int32 if items[0][0].dtype == "i32" else torch.float32
    outs = [torch.empty(p.n, dtype=tdt, device="cuda") for p, _ in items]
    for _ in range(reps):
        status, stats, _ = gbf.solve_batch(graphs, outs, mode=mode)
        assert status == gbf.OK
        for (p, e), gr, V, ref, st in zip(items, graphs, outs, refs, stats):
            Vh = V.cpu().numpy()
            bad = np.nonzero(Vh != ref["V"])[0]
            assert bad.size == 0, (p.name, e, bad[:8], Vh[bad[:8]], ref["V"][bad[:8]])
            pol, res = gr.policy()
            assert res == 0 and np.array_equal(pol, ref["policy"]), (p.name, e)
            assert st["status"] == gbf.OK
    for gr in graphs:
        gr.free()
    return stats


@pytest.mark.parametrize("mode", ["hostloop", "persistent"])
def test_batch_mixed_int32(mode):
    _case(f"batch mixed int32 {mode}")
    _check_batch(_small_mix("i32"), mode)


@pytest.mark.parametrize("mode", ["hostloop", "persistent"])
def test_batch_all_hybrid(mode):
    """A batch whose instances all use box successors with a reverse CSR."""
    _case(f"batch hybrid {mode}")
    _check_batch([(p, "box+rev") for p, _ in _small_mix("i32")], mode)


@pytest.mark.parametrize("mode", ["hostloop", "persistent"])
def test_batch_mixed_fp32(mode):
    _case(f"batch mixed fp32 {mode}")
    _check_batch(_small_mix("f32"), mode, precision="f32")


def test_batch_graph_replay():
    """The persistent batched solve with device outputs is captured in a HIP
    graph on the first call and replayed later; every replay is exact."""
    _case("batch graph replay")
    items = _small_mix("i32")
    stats = _check_batch(items, "persistent", reps=3)
    assert stats[0]["graph_used"] == 1


def test_batch_with_capped_instance():
    """An instance with a negative cycle stops at its own round cap; the
    others are unaffected."""
    _case("batch with negative cycle")
    import torch
    neg, _, _ = golden_io.load("negcycle.txt")
    fig, _, _ = golden_io.load("fig2_example.txt")
    items = [(fig, "csr"), (neg, "csr"), (synth.grid4d(synth.instance_seed(41, 0), dims=(10, 8, 5, 3), K=8), "csr")]
    graphs = [gbf.load_problem(p, encoding=e) for p, e in items]
    for mode in ("hostloop", "persistent"):
        outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p, _ in items]
        status, stats, _ = gbf.solve_batch(graphs, outs, mode=mode)
        assert status == gbf.ENEGCYCLE
        assert [s["status"] for s in stats] == [gbf.OK, gbf.ENEGCYCLE, gbf.OK]
        for i in (0, 2):
            assert np.array_equal(outs[i].cpu().numpy(), oracle.solve(items[i][0])["V"])
    for gr in graphs:
        gr.free()


@pytest.fixture(scope="module")
def batch64():
    """The 64-instance mix and the oracle's solution of every instance (the
    oracle's C calls release the interpreter lock, so threads run them in
    parallel)."""
    from concurrent.futures import ThreadPoolExecutor
    probs = synth.batch_mix(64, with_csr=False)
    with ThreadPoolExecutor(max_workers=8) as ex:
        refs = list(ex.map(oracle.solve, probs))
    return probs, refs


def _check64(probs, refs, graphs, outs, label):
    for i, (p, ref, gr, V) in enumerate(zip(probs, refs, graphs, outs)):
        Vh = V.cpu().numpy()
        bad = np.nonzero(Vh != ref["V"])[0]
        assert bad.size == 0, (label, i, p.name, bad[:8], Vh[bad[:8]], ref["V"][bad[:8]])
        pol, res = gr.policy()
        assert res == 0 and np.array_equal(pol, ref["policy"]), (label, i, p.name)


def test_batch64_vs_oracle(batch64):
    """The 64-instance mix (2-D 128x128, 3-D 48x48x24, 4-D up to
    40x40x24x10) with the library defaults: every instance bit-exact with
    the oracle (values and canonical policy), and equal to its single
    solve."""
    import torch
    probs, refs = batch64
    _case("batch64 defaults vs oracle")
    graphs = [gbf.load_problem(p, encoding="csr") for p in probs]
    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p in probs]
    status, stats, _ = gbf.solve_batch(graphs, outs)
    assert status == gbf.OK
    _check64(probs, refs, graphs, outs, "defaults")
    for i in range(0, 64, 7):
        st, s, Vs = graphs[i].solve()
        assert st == gbf.OK
        assert np.array_equal(Vs, refs[i]["V"]), probs[i].name
    for gr in graphs:
        gr.free()


def test_batch64_tuned_configuration_vs_oracle(batch64):
    """The configuration the autotuner picks for this mix on MI355X (box
    successors with a reverse CSR, host loop, 2 lanes per pair, 2048
    blocks): every instance bit-exact with the oracle."""
    import torch
    probs, refs = batch64
    _case("batch64 box+rev hostloop lanes=2 grid=2048 vs oracle")
    graphs = [gbf.load_problem(p, encoding="box+rev") for p in probs]
    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p in probs]
    status, stats, _ = gbf.solve_batch(graphs, outs, mode="hostloop", lanes=2, grid=2048)
    assert status == gbf.OK
    _check64(probs, refs, graphs, outs, "tuned")
    for gr in graphs:
        gr.free()


@pytest.mark.parametrize("encoding", ["csr", "box+rev"])
def test_batch64_graph_replays_vs_oracle(batch64, encoding):
    """The persistent form captured in a HIP graph and replayed: every
    replay bit-exact with the oracle on all 64 instances."""
    import torch
    probs, refs = batch64
    _case(f"batch64 persistent graph replays {encoding}")
    graphs = [gbf.load_problem(p, encoding=encoding) for p in probs]
    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p in probs]
    for rep in range(3):
        for V in outs:
            V.fill_(-7)
        status, stats, _ = gbf.solve_batch(graphs, outs, mode="persistent")
        assert status == gbf.OK
        assert stats[0]["graph_used"] == 1
        _check64(probs, refs, graphs, outs, f"graph-{encoding}-{rep}")
    for gr in graphs:
        gr.free()


def test_batch_after_free_and_reload():
    """Freeing the handles of a batch drops its captured graph: a new batch
    (whose handles may reuse the old addresses) is solved from scratch and
    exactly."""
    _case("batch after free and reload")
    import torch
    for rep in range(3):
        items = _small_mix("i32")[:3] if rep % 2 == 0 else _small_mix("i32")[2:]
        graphs = [gbf.load_problem(p, encoding=e) for p, e in items]
        outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p, _ in items]
        for _ in range(2):
            status, stats, _ = gbf.solve_batch(graphs, outs, mode="persistent")
            assert status == gbf.OK
            for (p, e), V in zip(items, outs):
                assert np.array_equal(V.cpu().numpy(), oracle.solve(p)["V"]), (rep, p.name, e)
        for gr in graphs:
            gr.free()
