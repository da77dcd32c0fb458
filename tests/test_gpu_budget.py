"""Memory-budgeted images (expand_box 3): the loader keeps the predecessor
images when they fit the budget and stays implicit otherwise; either way the
solve is exact against the oracle and the stats report the choice."""
import numpy as np
import pytest

import oracle
import paper_2001_06231_amd as gbf
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    gbf.lib()


@pytest.fixture(scope="module")
def grid():
    prob = synth.grid4d(synth.instance_seed(2, 23), dims=(12, 10, 6, 4), K=12)
    return prob, oracle.solve(prob)


def _run(prob, ref, encoding, **kw):
    gr = gbf.load_problem(prob, encoding=encoding, **kw)
    status, st, V = gr.solve()
    pol, res = gr.policy()
    gr.free()
    assert status == gbf.OK and res == 0
    assert np.array_equal(V, ref["V"]) and np.array_equal(pol, ref["policy"])
    return st


@pytest.mark.parametrize("budget,want", [(1 << 40, 2), (0, 2), (1, 1)])
def test_budget_choice(grid, budget, want):
    prob, ref = grid
    print(f"\n[case] budget {budget}", flush=True)
    st = _run(prob, ref, "box:budget", mem_budget=budget)
    assert st["enc_used"] == want


def test_enc_used_reported(grid):
    prob, ref = grid
    print("\n[case] enc_used", flush=True)
    assert _run(prob, ref, "csr")["enc_used"] == 0
    assert _run(prob, ref, "box")["enc_used"] == 1
    assert _run(prob, ref, "box+rev")["enc_used"] == 2
    # the implicit form holds less device memory than the one with images
    small = _run(prob, ref, "box:budget", mem_budget=1)["device_bytes"]
    big = _run(prob, ref, "box:budget", mem_budget=1 << 40)["device_bytes"]
    assert small < big
