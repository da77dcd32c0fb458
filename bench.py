"""Benchmark of the generalized Bellman-Ford solver on one MI355X.

One step = one full pass of the hot path on device-resident inputs: solve
(initialise W <- G, seed the frontier, every frontier round until it drains:
compact, relax, expand) plus extraction of the canonical controller with its
fixed-point residual.  Workload: the 4-D UAV-style grid 40x40x24x10
(384,000 cells), 12 inputs, int32 potential-form costs, explicit successor
lists (CSR).

Prints ONE JSON line.  `value` = edge relaxations (sum of |F(x,u)| over the
pairs the GPU evaluated) per second of step time.  `roofline` is for the
dominant kernel (the relax kernel in host-loop mode, the round kernel in
persistent mode): its algorithmic bytes per launch divided by its average
launch duration, both measured inside the timed steps with HIP events on the
solver's stream.  `traffic` is the measured HBM bytes per launch of that
kernel from the committed rocprofv3 counter summary, if the kernel source is
unchanged since it was taken.  `cpu_baseline` is the single-threaded CPU
oracle on the same instance.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "edge relaxations/sec + solve time, 4D 384k-cell graph; learned/batched vs plain"
KERNEL_SRC = os.path.join(ROOT, "paper_2001_06231_amd", "csrc", "gbf_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "relax_traffic_grid4d_384k.txt")


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_bytes(st, npairs, mode, rounds):
    """Bytes the method must move per solve (not cache behaviour):
    relax (CSR): 20 B per evaluated pair (list id 4, row bounds 8, cost 4,
    W(x) 4) + 8 B per edge (successor index 4, W(y) 4);
    expand: 8 B per expanded state (reverse-row bounds) + 5 B per marked
    predecessor pair (reverse entry 4, dirty byte 1);
    compact (part of the persistent and single-block kernels only): the dirty byte map
    is read once per round (npairs B) + 4 B per listed pair."""
    b = 20 * st["pair_evals"] + 8 * st["edge_relax"] + 8 * st["expansions"] + 5 * st["marks"]
    if mode in ("persistent", "single_block"):
        b += (rounds + 1) * npairs + 4 * st["pair_evals"]
    return b


def read_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None if it is missing or was taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash() or kv.get("kernel") != kernel:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _gen_learned(index):
    import synth
    return synth.learned_instance(index, with_csr=False)


def _gen_batch(i):
    import synth
    return synth.batch_instance(i, 64, with_csr=False)


def _gen_small(kind):
    import synth
    if kind == "grid2d":
        return synth.grid2d_small()
    return synth.grid4d(dtype="f32")


class _Done:
    """A finished job (generation without worker processes)."""

    def __init__(self, value):
        self.value = value

    def wait(self):
        pass

    def get(self):
        return self.value


def _median_solve(graph, reps, **kw):
    """Median-time solve over `reps` runs (after one warm-up): stats dict."""
    import numpy as np
    graph.solve(**kw)
    runs = [graph.solve(**kw)[1] for _ in range(reps)]
    med = float(np.median([r["solve_ms"] for r in runs]))
    best = min(runs, key=lambda r: abs(r["solve_ms"] - med))
    return dict(best, solve_ms=med)


def learned_compare(prob, params, untrained, reps=3):
    """Plain vs network-bucketed order on one instance: solve times, MLP
    inference time, relaxation counts, rounds; values compared bit for bit.
    `untrained` is the control network (initial weights)."""
    import torch

    import paper_2001_06231_amd as gbf
    from paper_2001_06231_amd import learn
    g = gbf.load_problem(prob, encoding="csr")
    Vp = torch.empty(prob.n, dtype=torch.int32, device="cuda")
    Vb = torch.empty_like(Vp)
    plain = _median_solve(g, reps, V_out=Vp)
    pol_p, _ = g.policy()
    tc = learn.target_centre(prob)
    out = {"instance": prob.name, "n_states": prob.n, "pairs": prob.npairs,
           "plain": {k: plain[k] for k in ("solve_ms", "rounds", "pair_evals", "edge_relax")}}
    for label, par in (("learned", params), ("untrained", untrained)):
        net = gbf.MLP(par)
        keys = torch.empty(prob.n, dtype=torch.int16, device="cuda")
        net.bucket_keys(prob.dims, tc, learn.SCALE, learn.WIDTH, keys=keys)  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        mlp_ms = []
        for _ in range(reps):
            e0.record()
            net.bucket_keys(prob.dims, tc, learn.SCALE, learn.WIDTH, keys=keys)
            e1.record()
            e1.synchronize()
            mlp_ms.append(e0.elapsed_time(e1))
        st = _median_solve(g, reps, V_out=Vb, order="buckets", bucket_key=keys)
        pol_b, res = g.policy()
        exact = bool(torch.equal(Vp, Vb)) and bool((pol_b == pol_p).all()) and res == 0
        out[label] = {"solve_ms": st["solve_ms"], "mlp_ms": sorted(mlp_ms)[len(mlp_ms) // 2],
                      "rounds": st["rounds"], "sweeps": st["sweeps"], "pair_evals": st["pair_evals"],
                      "edge_relax": st["edge_relax"], "fallback": st["fallback"], "bit_exact": exact}
        net.free()
    g.free()
    L, P = out["learned"], out["plain"]
    out["wall_speedup_incl_mlp"] = P["solve_ms"] / (L["solve_ms"] + L["mlp_ms"])
    out["relaxation_reduction"] = P["edge_relax"] / max(1, L["edge_relax"])
    return out


def batch_compare(probs, reps=3):
    """One batched solve of all instances, with the encoding and launch
    configuration picked by the autotuner, vs one plain solve per instance
    with the library defaults (wall time around the calls, device outputs);
    and the persistent form replayed from its HIP graph."""
    import numpy as np
    import torch

    import paper_2001_06231_amd as gbf
    from paper_2001_06231_amd import autotune
    t0 = time.time()
    tuned = autotune.autotune(probs, reps=2)
    tune_s = time.time() - t0
    graphs = [gbf.load_problem(p, encoding="csr") for p in probs]
    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p in probs]
    seq = [torch.empty_like(o) for o in outs]

    def wall(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t0))
        return float(np.median(ts)), r

    def sequential():
        return [gr.solve(v)[1] for gr, v in zip(graphs, seq)]

    seq_ms, seq_stats = wall(sequential)
    per_ms, (_, per_stats, _) = wall(lambda: gbf.solve_batch(graphs, outs, mode="persistent"))
    exact = all(bool(torch.equal(a, b)) for a, b in zip(outs, seq))
    if tuned["encoding"] != "csr":
        for gr in graphs:
            gr.free()
        graphs = [gbf.load_problem(p, encoding=tuned["encoding"]) for p in probs]
    bat_ms, (_, bat_stats, _) = wall(lambda: gbf.solve_batch(graphs, outs, mode=tuned["mode"], lanes=tuned["lanes"],
                                                             grid=tuned["grid"]))
    exact = exact and all(bool(torch.equal(a, b)) for a, b in zip(outs, seq))
    res = {"instances": len(probs), "n_states": int(sum(p.n for p in probs)),
           "pairs": int(sum(p.npairs for p in probs)),
           "sequential_ms": seq_ms, "batched_ms": bat_ms,
           "tuned": {k: tuned[k] for k in ("encoding", "mode", "lanes", "grid")}, "tune_s": tune_s,
           "persistent_graph_ms": per_ms, "graph_used": int(per_stats[0]["graph_used"]),
           "speedup": seq_ms / bat_ms,
           "edge_relax_batched": int(bat_stats[0]["edge_relax"]),
           "edge_relax_sequential": int(sum(s["edge_relax"] for s in seq_stats)),
           "rounds_batched": int(bat_stats[0]["rounds"]), "bit_exact": exact}
    for gr in graphs:
        gr.free()
    return res


def config_line(prob, encoding, reps=5):
    """Solve time, edge relaxations/s and device memory of one configuration."""
    import torch

    import paper_2001_06231_amd as gbf
    g = gbf.load_problem(prob, encoding=encoding)
    V = torch.empty(prob.n, dtype=torch.int32 if prob.dtype == "i32" else torch.float32, device="cuda")
    st = _median_solve(g, reps, V_out=V)
    g.free()
    return {"solve_ms": st["solve_ms"], "edge_relax_per_s": st["edge_relax"] / (st["solve_ms"] * 1e-3),
            "rounds": st["rounds"], "edge_relax": st["edge_relax"], "device_bytes": st["device_bytes"],
            "encoding": encoding}


def run(args, pool=None):
    import numpy as np
    import torch

    import paper_2001_06231_amd as gbf
    import synth

    jobs = {}
    if not args.no_extras:
        if pool is not None:
            jobs["learned"] = pool.apply_async(_gen_learned, (1000,))
            jobs["batch"] = pool.map_async(_gen_batch, range(64))
            jobs["grid2d"] = pool.apply_async(_gen_small, ("grid2d",))
            jobs["grid4d_f32"] = pool.apply_async(_gen_small, ("grid4d_f32",))
        else:
            jobs["learned"] = _Done(_gen_learned(1000))
            jobs["batch"] = _Done([_gen_batch(i) for i in range(64)])
            jobs["grid2d"] = _Done(_gen_small("grid2d"))
            jobs["grid4d_f32"] = _Done(_gen_small("grid4d_f32"))
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    t0 = time.time()
    prob = synth.grid4d()
    gen_s = time.time() - t0
    print(f"[bench] generated {prob.name}: n={prob.n} pairs={prob.npairs} m={prob.m} in {gen_s:.1f}s",
          file=sys.stderr, flush=True)
    if args.calib_copy:
        # a plain 256 MiB device copy: reference for the HBM byte counters
        x = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    t0 = time.time()
    graph = gbf.load_problem(prob, encoding="csr", stream=stream)
    torch.cuda.synchronize()
    load_s = time.time() - t0
    V = torch.empty(prob.n, dtype=torch.int32, device="cuda")
    pol = torch.empty(prob.n, dtype=torch.int32, device="cuda")
    # the other workloads are generated in worker processes; let them finish
    # first so that they do not compete with the host side of the timed loop
    for j in jobs.values():
        j.wait()

    def step():
        status, st, _ = graph.solve(V, mode=args.mode, lanes=args.lanes, grid=args.grid, profile=True)
        _, res = graph.policy(pol)
        if status != gbf.OK or res != 0:
            raise RuntimeError(f"solve failed: status={status} residual={res}")
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] {args.steps} steps in {elapsed:.3f}s", file=sys.stderr, flush=True)

    ms_per_step = 1e3 * elapsed / args.steps
    edges = float(np.mean([s["edge_relax"] for s in stats]))
    mode_used = {gbf.MODE_PERSISTENT: "persistent", gbf.MODE_SINGLE_BLOCK: "single_block"}.get(
        stats[0]["mode_used"], "hostloop")
    kernel = {"persistent": "k_persistent", "single_block": "k_single"}.get(mode_used, "k_relax")
    launches = sum(s["relax_launches"] for s in stats)
    kern_ms = sum(s["relax_ms"] for s in stats) / max(1, launches)
    total_bytes = sum(algorithmic_bytes(s, prob.npairs, mode_used, s["rounds"]) for s in stats)
    bytes_per_launch = total_bytes / max(1, launches)
    achieved = bytes_per_launch / (kern_ms * 1e-3) / 1e9
    traffic = read_traffic(kernel)
    out = {
        "metric": METRIC,
        "value": edges / (ms_per_step * 1e-3),
        "unit": "edge_relaxations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "grid4d 40x40x24x10 (x, y, heading, speed), 12 inputs, int32 potential-form costs, "
                        "CSR successors; one step = solve + canonical policy",
            "n_states": prob.n, "pairs": prob.npairs, "edges_m": prob.m,
            "parallelism": "single GPU",
        },
        "solve_ms": float(np.median([s["solve_ms"] for s in stats])),
        "rounds": int(np.median([s["rounds"] for s in stats])),
        "edge_relax_per_solve": edges,
        "pair_evals_per_solve": float(np.mean([s["pair_evals"] for s in stats])),
        "mode": mode_used,
        "lanes": int(stats[0]["lanes_used"]),
        "grid": int(stats[0]["grid_used"]),
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel_avg_ms": kern_ms,
            "launches_per_step": launches / args.steps,
            "algorithmic_bytes_per_launch": bytes_per_launch,
        },
        "load_s": load_s,
        "device_bytes": int(stats[0]["device_bytes"]),
        "kernel_source_sha256_16": kernel_source_hash(),
    }
    graph.free()
    if jobs:
        from paper_2001_06231_amd import learn
        extras = {}
        p2 = jobs["grid2d"].get()
        pf = jobs["grid4d_f32"].get()
        extras["grid2d_64x64_i32_csr"] = config_line(p2, "csr")
        extras["grid4d_384k_i32_box+rev"] = config_line(prob, "box+rev")
        extras["grid4d_384k_i32_box"] = config_line(prob, "box")
        extras["grid4d_384k_f32_csr"] = config_line(pf, "csr")
        extras["grid4d_384k_f32_box+rev"] = config_line(pf, "box+rev")
        extras["grid4d_384k_f32_box"] = config_line(pf, "box")
        # the same graph with the running cost on the edges, g(x,u) + h(x,y,u)
        extras["grid4d_384k_i32_csr_edge_costs"] = config_line(synth.with_edge_costs(prob, 34), "csr")
        print("[bench] configs done", file=sys.stderr, flush=True)
        out["configs"] = extras
        out["batch64"] = batch_compare(jobs["batch"].get())
        print("[bench] batch done", file=sys.stderr, flush=True)
        if os.path.exists(learn.WEIGHTS):
            out["learned"] = learned_compare(jobs["learned"].get(), learn.load_params(),
                                             learn.init_params(1))
        else:
            out["learned"] = {"skipped": "no trained weights"}
        print("[bench] learned done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_reps)
    return out


def learned_eval(args, pool):
    """Held-out evaluation of the trained network: instances 1000.. of the
    60x60x30x12 K=16 family.  Prints one JSON object."""
    import numpy as np
    import torch

    from paper_2001_06231_amd import learn
    torch.cuda.set_device(0)
    params = learn.load_params()
    untrained = learn.init_params(1)
    recs = []
    idx = list(range(1000, 1000 + args.learned_eval))
    gen = pool.imap(_gen_learned, idx) if pool is not None else map(_gen_learned, idx)
    for i, prob in zip(idx, gen):
        r = learned_compare(prob, params, untrained, reps=args.eval_reps)
        recs.append(r)
        print(f"[eval] {i}: plain {r['plain']['solve_ms']:.2f} ms / {r['plain']['edge_relax']:.3e} edges, "
              f"learned {r['learned']['solve_ms']:.2f} (+{r['learned']['mlp_ms']:.2f}) ms / "
              f"{r['learned']['edge_relax']:.3e}, untrained {r['untrained']['solve_ms']:.2f} ms, "
              f"exact {r['learned']['bit_exact'] and r['untrained']['bit_exact']}", file=sys.stderr, flush=True)

    def mean(f):
        return float(np.mean([f(r) for r in recs]))
    summary = {
        "instances": len(recs),
        "plain_solve_ms": mean(lambda r: r["plain"]["solve_ms"]),
        "learned_solve_ms": mean(lambda r: r["learned"]["solve_ms"]),
        "learned_mlp_ms": mean(lambda r: r["learned"]["mlp_ms"]),
        "untrained_solve_ms": mean(lambda r: r["untrained"]["solve_ms"]),
        "plain_edge_relax": mean(lambda r: r["plain"]["edge_relax"]),
        "learned_edge_relax": mean(lambda r: r["learned"]["edge_relax"]),
        "untrained_edge_relax": mean(lambda r: r["untrained"]["edge_relax"]),
        "plain_rounds": mean(lambda r: r["plain"]["rounds"]),
        "learned_rounds": mean(lambda r: r["learned"]["rounds"]),
        "all_bit_exact": all(r["learned"]["bit_exact"] and r["untrained"]["bit_exact"] for r in recs),
        "fallbacks": int(sum(r["learned"]["fallback"] + r["untrained"]["fallback"] for r in recs)),
    }
    summary["wall_speedup_incl_mlp"] = summary["plain_solve_ms"] / (summary["learned_solve_ms"] +
                                                                     summary["learned_mlp_ms"])
    summary["relaxation_reduction"] = summary["plain_edge_relax"] / summary["learned_edge_relax"]
    return {"summary": summary, "instances": recs}


def cpu_baseline(prob, reps):
    import numpy as np

    import oracle
    times, edges = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = oracle.solve(prob)
        times.append(time.perf_counter() - t0)
        edges.append(r["counters"]["edge_relax"])
    t = float(np.median(times))
    return {"value": float(np.median(edges)) / t, "unit": "edge_relaxations/s", "cores": 1, "kind": "oracle",
            "sample": f"the full 4-D 384k-cell instance, {reps} single-threaded solves (median); the oracle "
                      "counts its own relaxations (state frontier x all inputs)",
            "solve_s": t}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="auto", choices=["persistent", "hostloop", "single_block", "auto"])
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--calib-copy", action="store_true", help="run a 256 MiB device copy first (counter reference)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the main workload (no other configs, batch or learned comparison)")
    ap.add_argument("--learned-eval", type=int, default=0,
                    help="instead: evaluate the trained network on this many held-out instances")
    ap.add_argument("--eval-reps", type=int, default=3)
    ap.add_argument("--workers", type=int, default=8,
                    help="generator processes (1 = generate in this process, e.g. under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solver has no multi-GPU "
              "path", file=sys.stderr)
        sys.exit(2)
    # the generator workers are forked before the first GPU call
    pool = None
    if args.workers > 1 and (args.learned_eval or not args.no_extras):
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(args.workers)
    try:
        if args.learned_eval:
            print(json.dumps(learned_eval(args, pool)), flush=True)
        else:
            print(json.dumps(run(args, pool)), flush=True)
    finally:
        if pool is not None:
            pool.terminate()


if __name__ == "__main__":
    main()
