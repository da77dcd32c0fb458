"""Pins of the oracle's int32 reading of costs in R u {inf} (Sect. III-B;
Algorithm 1's backup g + sup W and strict test): INF = INT32_MAX, sums formed
exactly, a sum >= INT32_MAX is INF, a sum below -INT32_MAX clamps to
-INT32_MAX and is counted.  The expected values of the two fixtures were
worked out by hand from those rules (tests/golden/int32_limits*.txt).

Each plausible mistake in those branches is planted in a copy of the
oracle's source, compiled on the CPU, and must fail at least one fixture:
a sum wrapped around in 32 bits, a clamp at INT32_MIN instead of
-INT32_MAX, and a per-edge term h + W(y) that does not keep INF when W(y)
is INF.  (Testing the overflow with > instead of >= is not a mistake with
a different result: a sum of exactly INT32_MAX is stored as INF either way,
and INF is never a strict improvement.)"""
import numpy as np
import pytest

import oracle
from tests import golden_io

FIXTURES = ["int32_limits.txt", "int32_limits_edges.txt"]


def _check(name):
    prob, inputs, facts = golden_io.load(name)
    V, pol = golden_io.expected(facts, inputs, prob.n)
    r = oracle.solve(prob)
    ok = (r["status"] == oracle.OK and np.array_equal(r["V"], V) and np.array_equal(r["policy"], pol)
          and r["residual"] == 0)
    if facts.get("saturates", [["no"]])[0][0] == "yes":
        ok = ok and r["counters"]["saturations"] > 0
    return ok, r, V, pol


@pytest.mark.parametrize("name", FIXTURES)
def test_oracle_matches_hand_computed_values(name):
    ok, r, V, pol = _check(name)
    assert r["status"] == oracle.OK
    assert np.array_equal(r["V"], V), (r["V"], V)
    assert np.array_equal(r["policy"], pol), (r["policy"], pol)
    assert r["residual"] == 0
    assert r["counters"]["saturations"] > 0
    assert ok


def test_fixtures_exercise_both_limits():
    """Both fixtures hold INF values that come from an overflow (a state with
    finite successors and no finite backup) and values clamped at
    -INT32_MAX."""
    for name in FIXTURES:
        prob, inputs, facts = golden_io.load(name)
        V, _ = golden_io.expected(facts, inputs, prob.n)
        assert (V == golden_io.INF_I32).any() and (V == -golden_io.INF_I32).any(), name


MUTANTS = {
    # int32 sums wrapped around instead of formed in 64 bits
    "wraparound": [("int64_t s = (int64_t)g + (int64_t)m;",
                    "int64_t s = (int64_t)(int32_t)((uint32_t)g + (uint32_t)m);"),
                   ("int64_t s = (int64_t)g + m;", "int64_t s = (int64_t)(int32_t)((uint32_t)g + (uint32_t)m);")],
    # clamp at INT32_MIN instead of -INT32_MAX
    "int32_min_clamp": [("#define OR_LOW_I32 (-(int64_t)INT32_MAX)", "#define OR_LOW_I32 ((int64_t)INT32_MIN)")],
    # h + W(y) computed without keeping INF
    "edge_inf_slip": [("return (int64_t)w >= OR_INF_I32 ? OR_EDGE_INF_I64 : (int64_t)h + (int64_t)w;",
                       "return (int64_t)h + (int64_t)w;")],
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_planted_mistake_fails_a_fixture(mutant, tmp_path):
    src = oracle.source()
    for old, new in MUTANTS[mutant]:
        assert old in src, f"mutation site of {mutant} not found: {old}"
        src = src.replace(old, new)
    path = oracle.build_variant(src, str(tmp_path / f"liboracle_{mutant}.so"))
    with oracle.use_variant(path):
        results = [_check(name)[0] for name in FIXTURES]
    assert not all(results), f"the {mutant} mistake passes every int32 fixture"
    # the real oracle passes them all again
    assert all(_check(name)[0] for name in FIXTURES)
