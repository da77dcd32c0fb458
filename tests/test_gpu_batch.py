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
    return synth.batch_mix(64, with_csr=False)


def test_batch64_vs_single_solves(batch64):
    """The 64-instance mix (2-D 128x128, 3-D 48x48x24, 4-D up to
    40x40x24x10): the batched solve equals 64 single solves, and a sample is
    checked against the oracle."""
    import torch
    _case("batch64")
    graphs = [gbf.load_problem(p, encoding="csr") for p in batch64]
    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p in batch64]
    status, stats, _ = gbf.solve_batch(graphs, outs)
    assert status == gbf.OK
    for p, gr, V in zip(batch64, graphs, outs):
        st, s, Vs = gr.solve()
        assert st == gbf.OK
        assert np.array_equal(V.cpu().numpy(), Vs), p.name
    for i in (0, 16, 32):
        ref = oracle.solve(batch64[i])
        assert np.array_equal(outs[i].cpu().numpy(), ref["V"]), batch64[i].name
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
