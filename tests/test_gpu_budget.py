"""Memory-budgeted images (Sect. IV-B, VI-A: images kept in memory up to a
threshold, recomputed beyond it).  At load (expand_box 3) the predecessor
images are kept when they fit the budget, else the problem stays implicit;
during a solve (mem_floor_mib) they are released once the device's free
memory falls below a floor.  Every way the solve is exact against the
oracle and the stats report the representation."""
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


@pytest.mark.parametrize("wide", [False, True])
def test_images_dropped_under_memory_pressure(wide):
    """Predecessor images released during a solve once the device's free
    memory is below the floor (here a floor above the device's memory, so
    the first frontier-size check releases them): the rest of the solve and
    later solves search predecessors in the windows; values and policy stay
    the oracle's, and the handle holds less memory."""
    prob = synth.grid4d(synth.instance_seed(60, 1), dims=(20, 18, 10, 6), K=12)
    ref = oracle.solve(prob)
    print(f"\n[case] images dropped wide={wide}", flush=True)
    gr = gbf.load_problem(prob, encoding="box+rev", pair_ids64=wide)
    status, st0, V = gr.solve(mode="hostloop")
    assert status == gbf.OK and st0["enc_used"] == 2 and st0["images_dropped"] == 0
    status, st, V = gr.solve(mode="hostloop", mem_floor_mib=1 << 30)
    pol, res = gr.policy()
    assert status == gbf.OK and st["images_dropped"] == 1 and st["enc_used"] == 1, st
    assert st["device_bytes"] < st0["device_bytes"]
    assert res == 0 and np.array_equal(V, ref["V"]) and np.array_equal(pol, ref["policy"])
    status, st2, V2 = gr.solve(mode="hostloop")
    assert status == gbf.OK and st2["enc_used"] == 1 and st2["images_dropped"] == 0
    assert np.array_equal(V2, ref["V"])
    gr.free()
