"""Pins of the chained reward workload (Sect. VI-A: the second problem of
the mission flies to the hot spot with terminal cost G2 = V1, the value
function of the return problem, and a running cost that rewards the fire
region; here as per-edge costs R (1[x in fire] - 1[y in fire])).

The per-edge reward is a potential difference, so along any path it
telescopes to R 1[x0 in fire] - R 1[xT in fire], and inside the sup over
F(x,u) it splits into R 1[x in fire] and a per-successor shift of W.  So
the value function is V2 = R 1[fire] + V', with V' the value function of
the same system with per-pair costs only and terminal cost
G'(y) = G2(y) - R 1[y in fire] (INF where G2 is INF): a second oracle solve
on the per-pair path checks the per-edge path."""
import numpy as np
import pytest

import oracle
import synth

INF = synth.INF_I32


def _shifted(p2):
    import copy
    q = copy.copy(p2)
    q.g_edge = None
    G = np.asarray(p2.G, dtype=np.int64)
    f = p2.fire.astype(np.int64)
    q.G = np.where(G == INF, INF, G - p2.reward * f).astype(np.int32)
    return q


@pytest.fixture(scope="module", params=[(1, (16, 14, 8, 6), 24), (2, (12, 11, 6, 4), 24), (3, (12, 10, 6, 4), 5000)])
def chain(request):
    i, dims, R = request.param
    p1 = synth.grid4d(synth.instance_seed(2, 40 + i), dims=dims)
    r1 = oracle.solve(p1)
    p2 = synth.reward_problem(p1, r1["V"], 100 + i, reward=R)
    return p1, r1, p2, oracle.solve(p2)


def test_value_is_the_shifted_per_pair_value(chain):
    p1, r1, p2, r2 = chain
    assert r2["status"] == 0 and r2["residual"] == 0
    rs = oracle.solve(_shifted(p2))
    V = rs["V"].astype(np.int64)
    want = np.where(V == INF, INF, V + p2.reward * p2.fire.astype(np.int64))
    assert np.array_equal(r2["V"].astype(np.int64), want)


def test_chaining_only_lowers_values(chain):
    p1, r1, p2, r2 = chain
    V1, V2 = r1["V"], r2["V"]
    assert np.all((V2 <= V1) | (V1 == INF))
    assert np.array_equal(V2 == INF, V1 == INF)  # the same states can reach the airfield
    assert (V2 < V1).any() and (p2.g_edge < 0).any()


def test_fire_region_shape():
    p1 = synth.grid4d(synth.instance_seed(2, 45), dims=(20, 18, 8, 6))
    f = synth.fire_region(p1, 3)
    N = p1.dims
    x = np.nonzero(f)[0]
    c0, c1, c3 = x % N[0], (x // N[0]) % N[1], x // (N[0] * N[1] * N[2])
    assert c0.max() - c0.min() <= 5 and c1.max() - c1.min() <= 5 and c3.min() >= N[3] // 2
    assert not (f & (np.asarray(p1.G) == 0)).any() and not (f & (p1.avoid != 0)).any()
