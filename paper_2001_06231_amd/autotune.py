"""Autotuner: picks the successor encoding and the launch configuration for
a problem set (one problem, or the instances of a batch).

Every candidate encoding (explicit lists, box successors with predecessor
images, implicit boxes) is first screened with one solve at the library's
defaults; for the `finalists` fastest the set is loaded and gbf_tune
(include/gbf.h) times the launch configurations on the device (mode, lanes
per pair, relax grid and block, compaction grid); the fastest (encoding,
configuration) wins.  Results can be kept in a JSON cache keyed by the
shape of the set (grid dims, inputs and value type of every instance), so a
workload is tuned once.
"""
from __future__ import annotations

import hashlib
import json
import os

import time

from . import load_problem, solve_batch, tune

ENCODINGS = ("csr", "box+rev", "box")


def signature(probs) -> str:
    """Shape of a problem set: dims, inputs, value type and whether costs are
    per edge, per instance."""
    parts = [f"{tuple(int(d) for d in p.dims)}:{int(p.K)}:{p.dtype}"
             + (":edge" if getattr(p, "g_edge", None) is not None else "") for p in probs]
    return hashlib.sha1(";".join(parts).encode()).hexdigest()[:20]


def _measure(probs, encoding, reps, mode):
    graphs = [load_problem(p, encoding=encoding) for p in probs]
    try:
        return tune(graphs, reps=reps, mode=mode)
    finally:
        for g in graphs:
            g.free()


def _screen(probs, encoding, mode):
    """Solve time of the set in one encoding at the library's defaults (one
    untimed and one timed call)."""
    graphs = [load_problem(p, encoding=encoding) for p in probs]
    try:
        def run():
            if len(graphs) == 1:
                return graphs[0].solve(mode=mode)
            return solve_batch(graphs, mode=mode)
        run()
        t0 = time.perf_counter()
        run()
        return 1e3 * (time.perf_counter() - t0)
    finally:
        for g in graphs:
            g.free()


def _load_cache(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def autotune(probs, encodings=ENCODINGS, reps=3, cache=None, log=None, mode="auto", finalists=2):
    """Returns {"encoding", "mode", "lanes", "grid", "block", "compact_grid",
    "ms"} for the set, over every launch mode or within `mode`.  `cache`:
    path of a JSON file (read and updated), or None."""
    key = signature(probs) + ("" if mode == "auto" else f":{mode}")
    table = _load_cache(cache)
    if key in table:
        return table[key]
    best = None
    cands = []
    for enc in encodings:
        if enc != "csr" and any(getattr(p, "box_lo", None) is None for p in probs):
            continue  # no boxes: only explicit successor lists
        if enc != "csr" and any(getattr(p, "g_edge", None) is not None for p in probs):
            continue  # per-edge costs are attached to explicit successor lists
        cands.append(enc)
    if len(cands) > finalists:
        screen = {enc: _screen(probs, enc, mode) for enc in cands}
        if log:
            log("screen: " + ", ".join(f"{e} {t:.3f} ms" for e, t in screen.items()))
        cands = sorted(cands, key=lambda e: screen[e])[:finalists]
    for enc in cands:
        opts, ms = _measure(probs, enc, reps, mode)
        if log:
            log(f"tune {enc}: {opts} {ms:.3f} ms")
        if best is None or ms < best["ms"]:
            best = dict(opts, encoding=enc, ms=ms)
    if best is None:
        raise ValueError("no encoding could be tuned")
    if cache:
        table[key] = best
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best
