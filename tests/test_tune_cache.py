"""Host logic of the autotuner: signatures, encoding choice and the JSON
cache (the device timing is replaced by a stub)."""
import json

import synth
from paper_2001_06231_amd import autotune as T


def test_signature_depends_on_shape_only():
    a = synth.grid2d_small()
    b = synth.grid2d_small(seed=synth.instance_seed(1, 5))
    c = synth.grid3d(synth.instance_seed(1, 6), dims=(8, 6, 4), K=6)
    assert T.signature([a]) == T.signature([b])
    assert T.signature([a]) != T.signature([c])
    assert T.signature([a, c]) != T.signature([c, a])


def test_choice_and_cache(tmp_path, monkeypatch):
    calls = []

    def fake(probs, enc, reps, mode):
        calls.append(enc)
        return ({"mode": "hostloop", "lanes": 4 if enc == "csr" else 2, "grid": 2048},
                {"csr": 5.0, "box+rev": 4.0}[enc])

    monkeypatch.setattr(T, "_measure", fake)
    # screening at the defaults: the implicit boxes are slowest, so only the
    # two others are tuned in full
    monkeypatch.setattr(T, "_screen", lambda probs, enc, mode: {"csr": 6.0, "box+rev": 5.0, "box": 30.0}[enc])
    probs = [synth.grid2d_small()]
    cache = str(tmp_path / "tune.json")
    best = T.autotune(probs, cache=cache)
    assert best["encoding"] == "box+rev" and best["lanes"] == 2 and best["ms"] == 4.0
    assert sorted(calls) == ["box+rev", "csr"]
    table = json.load(open(cache))
    assert table[T.signature(probs)] == best
    again = T.autotune(probs, cache=cache)
    assert again == best and sorted(calls) == ["box+rev", "csr"]  # served from the cache


def test_lists_only_problem_skips_box(monkeypatch):
    prob = synth.explicit_problem(2, 1, [[1], [1]], [1, 0], [2**31 - 1, 0])
    seen = []
    monkeypatch.setattr(T, "_measure", lambda p, e, r, m: (seen.append(e) or ({"mode": "hostloop", "lanes": 4,
                                                                            "grid": 0}, 1.0)))
    assert T.autotune([prob])["encoding"] == "csr"
    assert seen == ["csr"]


def test_edge_costs_tune_only_lists(monkeypatch):
    """Problems with per-edge costs are tuned on explicit successor lists
    only, under a signature of their own."""
    base = synth.grid2d_small()
    prob = synth.with_edge_costs(base, 3)
    assert T.signature([prob]) != T.signature([base])
    seen = []

    def fake(probs, enc, reps, mode):
        seen.append(enc)
        return {"mode": "hostloop", "lanes": 4, "grid": 1024}, 1.0

    monkeypatch.setattr(T, "_measure", fake)
    best = T.autotune([prob])
    assert seen == ["csr"] and best["encoding"] == "csr"


def test_mode_restricted_tuning_has_its_own_cache_entry(tmp_path, monkeypatch):
    """Tuning within one launch mode passes the mode down and is cached
    under a key of its own, beside the unrestricted result."""
    seen = []

    def fake(probs, enc, reps, mode):
        seen.append(mode)
        return {"mode": "hostloop" if mode == "auto" else mode, "lanes": 2, "grid": 0}, 1.0

    monkeypatch.setattr(T, "_measure", fake)
    monkeypatch.setattr(T, "_screen", lambda probs, enc, mode: {"csr": 1.0, "box+rev": 2.0, "box": 3.0}[enc])
    probs = [synth.grid2d_small()]
    cache = str(tmp_path / "tune.json")
    a = T.autotune(probs, cache=cache)
    b = T.autotune(probs, cache=cache, mode="persistent")
    assert a["mode"] == "hostloop" and b["mode"] == "persistent"
    assert set(seen) == {"auto", "persistent"}
    table = json.load(open(cache))
    assert table[T.signature(probs)] == a and table[T.signature(probs) + ":persistent"] == b


def test_screening_keeps_the_finalists(monkeypatch):
    """With three encodings and two finalists, the slowest at the defaults
    is not tuned; with finalists=3 every encoding is."""
    seen, screened = [], []

    def screen(probs, enc, mode):
        screened.append(enc)
        return {"csr": 2.0, "box+rev": 1.0, "box": 9.0}[enc]

    def fake(probs, enc, reps, mode):
        seen.append(enc)
        return {"mode": "hostloop", "lanes": 4, "grid": 2048, "block": 512, "compact_grid": 0}, {"csr": 2.0, "box+rev": 1.0, "box": 0.5}[enc]

    monkeypatch.setattr(T, "_screen", screen)
    monkeypatch.setattr(T, "_measure", fake)
    probs = [synth.grid2d_small()]
    best = T.autotune(probs)
    assert sorted(screened) == ["box", "box+rev", "csr"] and sorted(seen) == ["box+rev", "csr"]
    assert best["encoding"] == "box+rev"
    seen.clear()
    screened.clear()
    best = T.autotune(probs, finalists=3)
    assert screened == [] and sorted(seen) == ["box", "box+rev", "csr"] and best["encoding"] == "box"
