"""GPU parity on the int32 limits (costs in R u {inf}, Sect. III-B; the
backup and strict test of Algorithm 1): sums that reach INT32_MAX are INF,
sums below -INT32_MAX clamp to -INT32_MAX, per-edge terms keep INF.  The
fixtures' hand-computed values pin the oracle (tests/test_oracle_int32_limits.py);
here the HIP path must match the oracle bit for bit in every solver mode,
in batches and in the bucket order, and must count saturations."""
import numpy as np
import pytest

import oracle
import paper_2001_06231_amd as gbf
from tests import golden_io

pytestmark = pytest.mark.gpu

FIXTURES = ["int32_limits.txt", "int32_limits_edges.txt"]
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


def _load(name):
    prob, inputs, facts = golden_io.load(name)
    V, pol = golden_io.expected(facts, inputs, prob.n)
    ref = oracle.solve(prob)
    assert np.array_equal(ref["V"], V) and np.array_equal(ref["policy"], pol)
    return prob, ref


def _exact(label, V, pol, res, ref):
    assert res == 0, (label, "residual", res)
    assert np.array_equal(np.asarray(V), ref["V"]), (label, np.asarray(V), ref["V"])
    assert np.array_equal(np.asarray(pol), ref["policy"]), (label, np.asarray(pol), ref["policy"])


@pytest.mark.parametrize("name", FIXTURES)
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("lanes", [1, 4])
def test_int32_limits_modes(name, mode, lanes):
    prob, ref = _load(name)
    _case(f"int32 limits {name} {mode} lanes={lanes}")
    gr = gbf.load_problem(prob)
    status, st, V = gr.solve(mode=mode, lanes=lanes)
    assert status == gbf.OK
    pol, res = gr.policy()
    _exact(f"{name}-{mode}", V, pol, res, ref)
    assert st["saturations"] > 0, st
    gr.free()


@pytest.mark.parametrize("mode", ["hostloop", "persistent"])
def test_int32_limits_in_a_batch(mode):
    """Both fixtures and the paper's example in one frontier (three graph
    replays in persistent mode)."""
    import torch
    _case(f"int32 limits batch {mode}")
    items = [_load(n) for n in FIXTURES]
    fig, _, _ = golden_io.load("fig2_example.txt")
    items.append((fig, oracle.solve(fig)))
    graphs = [gbf.load_problem(p) for p, _ in items]
    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p, _ in items]
    for rep in range(3 if mode == "persistent" else 1):
        status, stats, _ = gbf.solve_batch(graphs, outs, mode=mode)
        assert status == gbf.OK
        for (p, ref), gr, V, s in zip(items, graphs, outs, stats):
            pol, res = gr.policy()
            _exact(f"batch-{mode}-{rep}-{p.name}", V.cpu().numpy(), pol, res, ref)
        assert stats[0]["saturations"] > 0
    for gr in graphs:
        gr.free()


@pytest.mark.parametrize("name", FIXTURES)
def test_int32_limits_bucket_order(name):
    """The bucket order with keys that put every state in its own bucket, in
    reverse state order, and with all keys equal."""
    import torch
    prob, ref = _load(name)
    _case(f"int32 limits buckets {name}")
    gr = gbf.load_problem(prob)
    for keys in (np.arange(prob.n)[::-1].copy(), np.zeros(prob.n)):
        k = torch.tensor(keys.astype(np.int16), device="cuda")
        for span in (1, -1, 32):
            status, st, V = gr.solve(order="buckets", bucket_key=k, bucket_span=span)
            assert status == gbf.OK
            pol, res = gr.policy()
            _exact(f"buckets-{name}-{span}", V, pol, res, ref)
    gr.free()
