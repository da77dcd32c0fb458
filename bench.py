"""Benchmark of the generalized Bellman-Ford solver on one MI355X.

One step = one full pass of the hot path on device-resident inputs: solve
(initialise W <- G, seed the frontier, every frontier round until it drains:
compact, relax, expand) plus extraction of the canonical controller with its
fixed-point residual.  Main workload: the 4-D UAV-style grid 40x40x24x10
(384,000 cells), 12 inputs, int32 potential-form costs, explicit successor
lists (CSR).

Prints ONE JSON line.  `value` = edge relaxations (sum of |F(x,u)| over the
pairs the GPU evaluated) per second of step time.  Every workload (the main
line, each entry of `configs`, `batch64`, `learned`) carries:
  - `roofline` of its dominant kernel (the relax kernel in host-loop mode,
    the round kernel in persistent or single-workgroup mode): algorithmic
    bytes per launch (the counters of the solves times the per-unit bytes
    below) over the kernel's average launch duration, measured with HIP
    events on the solver's stream around every launch;
  - `cpu_baseline`: the single-threaded CPU oracle, pinned to one host core
    (its own worker process), on the same workload or a stated sample.
Algorithmic bytes per unit (what the method must move, not cache behaviour):
  relax: 20 B per evaluated pair (list id 4, row bounds 8, cost 4, W(x) 4)
         + per successor 8 B (CSR: index 4 + W(y) 4), 4 B (box successors:
         W(y)), 12 B (CSR with per-edge costs: index, h, W(y));
  expand: 8 B per improved state (reverse-row bounds) + 8 B per predecessor
         pair or box candidate visited (reverse entry 4 + frontier word 4);
  compact (inside the persistent and single-workgroup kernels only): the
         frontier read and cleared once per round, nK/4 B, + 4 B per listed
         pair.
`traffic` is the measured HBM bytes per launch of the main line's kernel
from the committed rocprofv3 counter summary, if the kernel source is
unchanged since it was taken.
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
PER_EDGE_BYTES = {"csr": 8, "box->csr": 8, "box": 4, "box+rev": 4, "box:budget": 4, "csr_edge": 12}
KERNEL_OF_MODE = {"persistent": "k_persistent", "single_block": "k_single", "hostloop": "k_relax"}
REWARD_SEED = 7  # fire region of the chained reward workload


def kernel_source_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_bytes(st, npairs, per_edge, mode):
    """Bytes the method must move in one solve, from its counters (see the
    module docstring)."""
    b = 20 * st["pair_evals"] + per_edge * st["edge_relax"] + 8 * st["expansions"] + 8 * st["marks"]
    if mode in ("persistent", "single_block"):
        b += (st["rounds"] + 1) * npairs / 4 + 4 * st["pair_evals"]
    return b


def mode_name(st):
    import paper_2001_06231_amd as gbf
    return {gbf.MODE_PERSISTENT: "persistent", gbf.MODE_SINGLE_BLOCK: "single_block"}.get(st["mode_used"],
                                                                                         "hostloop")


def roofline(stats, npairs, per_edge, small_lds=False):
    """Roofline object of the dominant kernel over solves run with
    profile=True (HIP events around every launch of that kernel)."""
    mode = mode_name(stats[0])
    kernel = KERNEL_OF_MODE[mode]
    if mode == "single_block" and small_lds:
        kernel = "k_small"  # the single-workgroup solver with V and the frontiers in LDS
    launches = sum(s["relax_launches"] for s in stats)
    kern_ms = sum(s["relax_ms"] for s in stats) / max(1, launches)
    nbytes = sum(algorithmic_bytes(s, npairs, per_edge, mode) for s in stats) / max(1, launches)
    achieved = nbytes / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else 0.0
    return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel_avg_ms": kern_ms,
            "launches_per_solve": launches / len(stats), "algorithmic_bytes_per_launch": nbytes}


AC_SRC = os.path.join(ROOT, "paper_2001_06231_amd", "csrc", "gbf_aircraft.hip")
AC_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "aircraft_traffic_200x70x75x135_k35.txt")


def read_ac_traffic():
    """HBM bytes per relax step (k_ac_relax + k_ac_expand) of the aircraft
    mission's problem 1 on the paper's grid, raw counters, from the
    committed summary; None if missing or taken on another source."""
    if not os.path.exists(AC_TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(AC_TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    with open(AC_SRC, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    if kv.get("aircraft_source_sha256_16") != h:
        return None
    try:
        return float(kv["hbm_bytes_raw"]) / float(kv["relax_launches"])
    except (KeyError, ValueError, ZeroDivisionError):
        return None


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


# ---------------------------------------------------------------- inputs
def make_problem(kind):
    """The synthetic inputs of every workload, by name."""
    import synth
    if kind == "grid2d":
        return synth.grid2d_small()
    if kind == "grid4d_i32":
        return synth.grid4d()
    if kind == "grid4d_f32":
        return synth.grid4d(dtype="f32")
    if kind == "grid4d_i32_edge":
        return synth.with_edge_costs(synth.grid4d(), 34)
    if kind.startswith("batch:"):
        return synth.batch_instance(int(kind[6:]), 64, with_csr=False)
    if kind.startswith("learned:"):
        return synth.learned_instance(int(kind[8:]), with_csr=False)
    raise ValueError(kind)


class _Done:
    """A finished job (when no worker processes are used)."""

    def __init__(self, value):
        self.value = value

    def wait(self):
        pass

    def get(self):
        return self.value


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0))}


# ---------------------------------------------------------------- CPU oracle
def cpu_job(spec):
    """Runs in a worker process pinned to one host core: times the oracle's
    whole solve call (its own predecessor lists, Algorithm 1 and the policy
    pass); generating the input is outside the clock."""
    label, kinds, reps, precision, core = spec
    if core is not None:
        os.sched_setaffinity(0, {core})
    import numpy as np

    import oracle
    import synth
    oracle.lib()
    probs = []
    for k in kinds:
        if k.startswith("aircraft"):
            # "aircraftS:<grid>": problem S of the aircraft mission, its
            # explicit images built off the clock (problem 2 takes the
            # oracle's V_1, also solved off the clock)
            import oracle.aircraft as OA
            import synth.aircraft as SA
            stage, grid = int(k[8]), k.split(":")[1]
            make = getattr(SA, grid)
            G = None
            if stage == 2:
                G = oracle.solve(OA.problem(make(1)), precision="f32")["V"]
            probs.append(OA.problem(make(stage), G=G))
        elif k.startswith("reward:"):
            # the second problem of the chained mission: its terminal cost is
            # the oracle's value function of the first (solved off the clock)
            p1 = make_problem(k[7:])
            probs.append(synth.reward_problem(p1, oracle.solve(p1)["V"], REWARD_SEED))
        else:
            probs.append(make_problem(k))
    times, edges, pairs = [], [], []
    for _ in range(reps):
        t_sum, e_sum, p_sum = 0.0, 0, 0
        for p in probs:
            t0 = time.perf_counter()
            r = oracle.solve(p, precision=precision)
            t_sum += time.perf_counter() - t0
            e_sum += r["counters"]["edge_relax"]
            p_sum += r["counters"]["pair_evals"]
        times.append(t_sum)
        edges.append(e_sum)
        pairs.append(p_sum)
    t = float(np.median(times))
    e = float(np.median(edges))
    return label, {"value": e / t, "unit": "edge_relaxations/s", "cores": 1, "kind": "oracle",
                   "solve_s": t, "edge_relax": e, "pair_evals": float(np.median(pairs)),
                   "pinned_core": core, "reps": reps}


CPU_SAMPLES = {
    # label: (problem kinds, repetitions, precision, description)
    "main": (["grid4d_i32"], 3, None, "the full 4-D 40x40x24x10 int32 instance, median of 3 solves"),
    "grid2d_64x64_i32_csr": (["grid2d"], 5, None, "the full 2-D 64x64 instance, median of 5 solves"),
    "grid4d_384k_f32": (["grid4d_f32"], 1, "f32", "the full 4-D 40x40x24x10 fp32 instance, one solve with the "
                                                  "single-precision operator (encoding-independent)"),
    "grid4d_384k_i32_csr_edge_costs": (["grid4d_i32_edge"], 1, None,
                                       "the full 4-D 40x40x24x10 int32 instance with per-edge costs, one solve"),
    "grid4d_384k_i32_reward_chain": (["reward:grid4d_i32"], 1, None,
                                     "the second problem of the chained mission on the 4-D 40x40x24x10 grid "
                                     "(per-edge reward for the fire region, G2 = the oracle's V1 of the main "
                                     "instance), one solve; the first problem is solved off the clock"),
    "batch64": ([f"batch:{i}" for i in range(0, 64, 4)], 1, None,
                "16 of the 64 batch instances (every 4th: 4 2-D, 4 3-D, 8 4-D), one solve each; the rate is "
                "their summed relaxations over their summed solve time"),
    "learned": (["learned:1000"], 1, None, "held-out instance 1000 (60x60x30x12, K=16), one solve"),
    "aircraft_mission": (["aircraft1:medium", "aircraft2:medium"], 1, "f32",
                         "the aircraft mission on the 24x12x24x12 grid (82,944 cells, 35 inputs, landing within 90 "
                         "degrees): problem 1, then problem 2 with the oracle's V1, each on the oracle's own "
                         "explicit images (built off the clock), single-precision operator, one solve each"),
}


def start_cpu_jobs(pool, labels):
    cores = sorted(os.sched_getaffinity(0))
    # leave the lowest core to the process that drives the GPU
    usable = cores[1:] if len(cores) > len(labels) else cores
    specs = []
    for i, lab in enumerate(labels):
        kinds, reps, prec, _ = CPU_SAMPLES[lab]
        specs.append((lab, kinds, reps, prec, usable[(len(usable) - 1 - i) % len(usable)]))
    if pool is None:
        return _Done([cpu_job(s) for s in specs])
    return pool.map_async(cpu_job, specs)


def attach_cpu(res, cpu_results, label, info):
    if label in cpu_results:
        c = dict(cpu_results[label])
        c["sample"] = CPU_SAMPLES[label][3] + ("; the oracle counts its own relaxations (state frontier x all "
                                               "inputs), so the rate is throughput, not a comparison of counts")
        c.update(info)
        res["cpu_baseline"] = c


# ---------------------------------------------------------------- GPU legs
def measure(graph, prob, encoding, reps=5, V=None, **kw):
    """Median solve time over `reps` solves after one warm-up, edge
    relaxations/s, and the roofline of the dominant kernel (the same solves
    run with per-launch events)."""
    import numpy as np
    import torch
    if V is None:
        V = torch.empty(prob.n, dtype=torch.int32 if prob.dtype == "i32" else torch.float32, device="cuda")
    graph.solve(V, **kw)
    runs = [graph.solve(V, **kw)[1] for _ in range(reps)]
    med = float(np.median([r["solve_ms"] for r in runs]))
    best = min(runs, key=lambda r: abs(r["solve_ms"] - med))
    prof = [graph.solve(V, profile=True, **kw)[1] for _ in range(reps)]
    per_edge = PER_EDGE_BYTES["csr_edge" if getattr(prob, "g_edge", None) is not None else encoding]
    return {"solve_ms": med, "edge_relax_per_s": best["edge_relax"] / (med * 1e-3), "rounds": best["rounds"],
            "pair_evals": best["pair_evals"], "edge_relax": best["edge_relax"],
            "device_bytes": best["device_bytes"], "encoding": encoding, "mode": mode_name(best),
            "roofline": roofline(prof, prob.npairs, per_edge,
                                 small_lds=encoding in ("csr", "box+rev") and prob.npairs <= 16384 and prob.n <= 6144)}


def config_line(prob, encoding, reps=5):
    import paper_2001_06231_amd as gbf
    g = gbf.load_problem(prob, encoding=encoding)
    try:
        return measure(g, prob, encoding, reps)
    finally:
        g.free()


def learned_compare(prob, params, untrained, reps=3):
    """Plain vs network-bucketed order on one instance: solve times, MLP
    inference time, relaxation counts, rounds; values compared bit for bit
    (GPU plain order against GPU bucket order; both are checked against the
    oracle in the tests)."""
    import torch

    import paper_2001_06231_amd as gbf
    from paper_2001_06231_amd import learn
    g = gbf.load_problem(prob, encoding="csr")
    Vp = torch.empty(prob.n, dtype=torch.int32, device="cuda")
    Vb = torch.empty_like(Vp)
    plain = measure(g, prob, "csr", reps, V=Vp)
    g.solve(Vp)
    pol_p, _ = g.policy()
    tc = learn.target_centre(prob)
    out = {"instance": prob.name, "n_states": prob.n, "pairs": prob.npairs, "plain": plain}
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
        st = measure(g, prob, "csr", reps, V=Vb, order="buckets", bucket_key=keys)
        g.solve(Vb, order="buckets", bucket_key=keys)
        pol_b, res = g.policy()
        exact = bool(torch.equal(Vp, Vb)) and bool((pol_b == pol_p).all()) and res == 0
        last = g.solve(Vb, order="buckets", bucket_key=keys)[1]
        st.update({"mlp_ms": sorted(mlp_ms)[len(mlp_ms) // 2], "sweeps": last["sweeps"],
                   "fallback": last["fallback"], "bit_exact_vs_plain_gpu": exact})
        out[label] = st
        net.free()
    g.free()
    L, P = out["learned"], out["plain"]
    out["wall_speedup_incl_mlp"] = P["solve_ms"] / (L["solve_ms"] + L["mlp_ms"])
    out["relaxation_reduction"] = P["edge_relax"] / max(1, L["edge_relax"])
    out["roofline"] = L["roofline"]
    return out


def batch_compare(probs, reps=3):
    """One batched solve of the 64 instances in the encoding and launch
    configuration the autotuner picks, against 64 sequential plain solves
    (library defaults) in the same encoding and in CSR; in the chosen
    encoding also the best host-loop configuration against the best
    persistent one replayed from its HIP graph (each tuned within its own
    mode), so the graph form is compared like for like; wall time around the
    calls (device outputs)."""
    import numpy as np
    import torch

    import paper_2001_06231_amd as gbf
    from paper_2001_06231_amd import autotune
    t0 = time.time()
    tuned = autotune.autotune(probs, reps=2)
    tune_s = time.time() - t0

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

    outs = [torch.empty(p.n, dtype=torch.int32, device="cuda") for p in probs]
    seq = [torch.empty_like(o) for o in outs]
    res = {"instances": len(probs), "n_states": int(sum(p.n for p in probs)),
           "pairs": int(sum(p.npairs for p in probs)),
           "tuned": {k: tuned.get(k, 0) for k in ("encoding", "mode", "lanes", "grid", "block", "compact_grid")},
           "tune_s": tune_s}
    exact = True

    def same():
        return all(bool(torch.equal(a, b)) for a, b in zip(outs, seq))
    for enc in dict.fromkeys(["csr", tuned["encoding"]]):
        graphs = [gbf.load_problem(p, encoding=enc) for p in probs]
        seq_ms, seq_stats = wall(lambda: [gr.solve(v)[1] for gr, v in zip(graphs, seq)])
        res[f"sequential_{enc}_ms"] = seq_ms
        res[f"edge_relax_sequential_{enc}"] = int(sum(s["edge_relax"] for s in seq_stats))
        per_ms, (_, per_stats, _) = wall(lambda: gbf.solve_batch(graphs, outs, mode="persistent"))
        exact = exact and same()
        res[f"persistent_graph_{enc}_ms"] = per_ms
        res[f"graph_used_{enc}"] = int(per_stats[0]["graph_used"])
        if enc == tuned["encoding"]:
            kw = dict(mode=tuned["mode"], lanes=tuned["lanes"], grid=tuned["grid"], block=tuned.get("block", 0),
                      compact_grid=tuned.get("compact_grid", 0))
            bat_ms, (_, bat_stats, _) = wall(lambda: gbf.solve_batch(graphs, outs, **kw))
            exact = exact and same()
            prof = [gbf.solve_batch(graphs, outs, profile=True, **kw)[1][0] for _ in range(reps)]
            per_edge = PER_EDGE_BYTES[enc]
            res["roofline"] = roofline(prof, res["pairs"], per_edge)
            res["batched_ms"] = bat_ms
            res["edge_relax_batched"] = int(bat_stats[0]["edge_relax"])
            res["rounds_batched"] = int(bat_stats[0]["rounds"])
            res["edge_relax_per_s_batched"] = bat_stats[0]["edge_relax"] / (bat_ms * 1e-3)
            # like for like: each launch form at its own best configuration
            forms = {}
            for mode in ("hostloop", "persistent"):
                o, _ = gbf.tune(graphs, reps=2, mode=mode)
                ms, (_, fst, _) = wall(lambda: gbf.solve_batch(graphs, outs, **o))
                exact = exact and same()
                forms[mode] = {"ms": ms, "lanes": int(o["lanes"]), "block": int(o["block"]), "grid": int(fst[0]["grid_used"]),
                               "graph_used": int(fst[0]["graph_used"]), "barrier_ms": fst[0]["barrier_ms"]}
            res["best_hostloop"] = forms["hostloop"]
            res["best_persistent_graph"] = forms["persistent"]
            res["graph_speedup_over_hostloop"] = forms["hostloop"]["ms"] / forms["persistent"]["ms"]
        for gr in graphs:
            gr.free()
    res["speedup_same_encoding"] = res[f"sequential_{tuned['encoding']}_ms"] / res["batched_ms"]
    res["speedup_vs_sequential_csr"] = res["sequential_csr_ms"] / res["batched_ms"]
    res["bit_exact_vs_sequential_gpu"] = exact
    return res


def run(args, pool=None):
    import numpy as np
    import torch

    import paper_2001_06231_amd as gbf

    info = host_info()
    jobs = {}
    cpu_labels = []
    if not args.no_cpu:
        cpu_labels = ["main"] + ([] if args.no_extras else
                                 ["grid2d_64x64_i32_csr", "grid4d_384k_f32", "grid4d_384k_i32_csr_edge_costs",
                                  "grid4d_384k_i32_reward_chain", "batch64", "learned"]
                                 + ([] if args.no_aircraft else ["aircraft_mission"]))
        jobs["cpu"] = start_cpu_jobs(pool, cpu_labels)
    if not args.no_extras:
        for kind in ("grid2d", "grid4d_f32", "grid4d_i32_edge", "learned:1000"):
            jobs[kind] = pool.apply_async(make_problem, (kind,)) if pool is not None else _Done(make_problem(kind))
        jobs["batch"] = (pool.map_async(make_problem, [f"batch:{i}" for i in range(64)]) if pool is not None
                         else _Done([make_problem(f"batch:{i}") for i in range(64)]))
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    t0 = time.time()
    prob = make_problem("grid4d_i32")
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
    for k, j in jobs.items():
        if k != "cpu":
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
    rl = roofline(stats, prob.npairs, PER_EDGE_BYTES["csr"])
    rl["traffic"] = read_traffic(rl["kernel"])
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
        "mode": mode_name(stats[0]),
        "lanes": int(stats[0]["lanes_used"]),
        "grid": int(stats[0]["grid_used"]),
        "roofline": rl,
        "load_s": load_s,
        "device_bytes": int(stats[0]["device_bytes"]),
        "kernel_source_sha256_16": kernel_source_hash(),
    }
    V1 = V.cpu().numpy()  # the main instance's value function: G2 of the chained reward workload
    graph.free()
    if not args.no_extras:
        import synth
        from paper_2001_06231_amd import learn
        extras = {}
        p2 = jobs["grid2d"].get()
        pf = jobs["grid4d_f32"].get()
        pe = jobs["grid4d_i32_edge"].get()
        extras["grid2d_64x64_i32_csr"] = config_line(p2, "csr")
        extras["grid4d_384k_i32_box+rev"] = config_line(prob, "box+rev")
        extras["grid4d_384k_i32_box"] = config_line(prob, "box")
        extras["grid4d_384k_f32_csr"] = config_line(pf, "csr")
        extras["grid4d_384k_f32_box+rev"] = config_line(pf, "box+rev")
        extras["grid4d_384k_f32_box"] = config_line(pf, "box")
        # the same graph with the running cost on the edges, g(x,u) + h(x,y,u)
        extras["grid4d_384k_i32_csr_edge_costs"] = config_line(pe, "csr")
        # the chained mission (Sect. VI-A): fly to the fire region with the
        # return problem's value function as terminal cost
        pr = synth.reward_problem(prob, V1, REWARD_SEED)
        extras["grid4d_384k_i32_reward_chain"] = config_line(pr, "csr")
        extras["grid4d_384k_i32_reward_chain"].update(
            {"fire_cells": int(pr.fire.sum()), "reward": int(pr.reward),
             "negative_edges": int((pr.g_edge < 0).sum()), "first_problem_solve_ms": out["solve_ms"]})
        print("[bench] configs done", file=sys.stderr, flush=True)
        out["configs"] = extras
        out["batch64"] = batch_compare(jobs["batch"].get())
        print("[bench] batch done", file=sys.stderr, flush=True)
        if os.path.exists(learn.WEIGHTS):
            out["learned"] = learned_compare(jobs["learned:1000"].get(), learn.load_params(), learn.init_params(1))
        else:
            out["learned"] = {"skipped": "no trained weights"}
        print("[bench] learned done", file=sys.stderr, flush=True)
        if not args.no_aircraft:
            import synth.aircraft as SA
            out["configs"]["aircraft_mission_200x70x75x135_k35"] = aircraft_mission(
                SA.PAPER_DIMS, samples=500, timed_solve=False,
                log=lambda m: print(f"[bench] aircraft {m}", file=sys.stderr, flush=True))
    if "cpu" in jobs:
        cpu = dict(jobs["cpu"].get())
        print("[bench] cpu baselines done", file=sys.stderr, flush=True)
        attach_cpu(out, cpu, "main", info)
        if not args.no_extras:
            attach_cpu(out["configs"]["grid2d_64x64_i32_csr"], cpu, "grid2d_64x64_i32_csr", info)
            for k in ("grid4d_384k_f32_csr", "grid4d_384k_f32_box+rev", "grid4d_384k_f32_box"):
                attach_cpu(out["configs"][k], cpu, "grid4d_384k_f32", info)
            for k in ("grid4d_384k_i32_box+rev", "grid4d_384k_i32_box"):
                attach_cpu(out["configs"][k], cpu, "main", info)
            attach_cpu(out["configs"]["grid4d_384k_i32_csr_edge_costs"], cpu, "grid4d_384k_i32_csr_edge_costs", info)
            attach_cpu(out["configs"]["grid4d_384k_i32_reward_chain"], cpu, "grid4d_384k_i32_reward_chain", info)
            attach_cpu(out["batch64"], cpu, "batch64", info)
            if "plain" in out["learned"]:
                attach_cpu(out["learned"], cpu, "learned", info)
            if "aircraft_mission_200x70x75x135_k35" in out["configs"]:
                attach_cpu(out["configs"]["aircraft_mission_200x70x75x135_k35"], cpu, "aircraft_mission", info)
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
    idx = [f"learned:{i}" for i in range(1000, 1000 + args.learned_eval)]
    gen = pool.imap(make_problem, idx) if pool is not None else map(make_problem, idx)
    for i, prob in zip(idx, gen):
        r = learned_compare(prob, params, untrained, reps=args.eval_reps)
        recs.append(r)
        print(f"[eval] {i}: plain {r['plain']['solve_ms']:.2f} ms / {r['plain']['edge_relax']:.3e} edges, "
              f"learned {r['learned']['solve_ms']:.2f} (+{r['learned']['mlp_ms']:.2f}) ms / "
              f"{r['learned']['edge_relax']:.3e}, untrained {r['untrained']['solve_ms']:.2f} ms "
              f"(fallback {r['untrained']['fallback']}), "
              f"exact {r['learned']['bit_exact_vs_plain_gpu'] and r['untrained']['bit_exact_vs_plain_gpu']}",
              file=sys.stderr, flush=True)

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
        "all_bit_exact": all(r["learned"]["bit_exact_vs_plain_gpu"] and r["untrained"]["bit_exact_vs_plain_gpu"]
                             for r in recs),
        "fallbacks_learned": int(sum(r["learned"]["fallback"] for r in recs)),
        "fallbacks_untrained": int(sum(r["untrained"]["fallback"] for r in recs)),
    }
    summary["wall_speedup_incl_mlp"] = summary["plain_solve_ms"] / (summary["learned_solve_ms"] +
                                                                     summary["learned_mlp_ms"])
    summary["relaxation_reduction"] = summary["plain_edge_relax"] / summary["learned_edge_relax"]
    summary["untrained_over_plain"] = summary["untrained_solve_ms"] / summary["plain_solve_ms"]
    return {"summary": summary, "instances": recs}


def paper_scale_run(args):
    """The paper-scale grid (200x70x75x135 = 141.75 M cells, 35 inputs, 4.96 G
    pairs; synth.paper_scale): generated on the device, loaded with 64-bit
    pair ids (box successors with a reverse CSR, or implicit boxes), solved
    once with per-launch events (roofline) and once for the solve time; the
    GPU's fixed-point residual over every state, and the oracle's own
    one-application-of-P check at sampled states.  Prints one JSON object."""
    import numpy as np
    import torch

    import oracle
    import paper_2001_06231_amd as gbf
    from synth import paper_scale as ps

    def log(msg):
        print(f"[paper-scale] {msg}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    m = ps.meta()
    n, K = m["n"], ps.K
    t0 = time.time()
    box, g, G, av = ps.build(m, "cuda", log=log)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    av_host = av.cpu().numpy()
    log(f"generated n={n} pairs={n * K} in {gen_s:.1f}s")
    t0 = time.time()
    gr = gbf.load_graph(n, K, G, g, encoding="box", dims=ps.DIMS, box=box, avoid=av,
                        expand_box=args.paper_expand, mem_budget=0)
    torch.cuda.synchronize()
    load_s = time.time() - t0
    del box, g, G, av
    torch.cuda.empty_cache()
    log(f"loaded in {load_s:.1f}s")
    V = torch.empty(n, dtype=torch.int32, device="cuda")
    status, st_prof, _ = gr.solve(V, profile=True)
    log(f"profiled solve: status {status} {st_prof['solve_ms']:.0f} ms rounds {st_prof['rounds']}")
    status, st, _ = gr.solve(V)
    log(f"solve: status {status} {st['solve_ms']:.0f} ms")
    pol = torch.empty(n, dtype=torch.int32, device="cuda")
    _, res = gr.policy(pol)
    Vh = V.cpu().numpy()
    enc = PER_EDGE_BYTES["box+rev" if st["enc_used"] == 2 else "box"]
    rl = roofline([st_prof], n * K, enc)
    gr.free()
    t0 = time.time()
    xs = ps.sample_states(args.paper_samples, m)
    rows_b, rows_g = [], []
    for i0 in range(0, xs.size, 100000):
        xi = xs[i0:i0 + 100000]
        pid = (xi[:, None] * K + np.arange(K)[None, :]).reshape(-1)
        b, c = ps.pair_rows(torch.from_numpy(pid), m)
        rows_b.append(b.numpy().view(np.uint64))
        rows_g.append(c.numpy())
    Gs, _ = ps.state_rows(torch.from_numpy(xs), m)
    bad, first = oracle.residual_box_sample(ps.DIMS, K, xs, np.concatenate(rows_b), np.concatenate(rows_g),
                                            Gs.numpy(), av_host, Vh)
    check_s = time.time() - t0
    log(f"oracle check at {xs.size} states: {bad} mismatches in {check_s:.1f}s")
    fin = Vh != gbf.INF_I32
    return {
        "workload": "paper-scale grid 200x70x75x135 (141.75 M cells), 35 inputs, int32 potential-form costs, "
                    "box successors, 64-bit pair ids",
        "n_states": n, "pairs": n * K, "status": int(status), "enc_used": int(st["enc_used"]),
        "device_bytes": int(st["device_bytes"]),
        "gen_s": gen_s, "load_s": load_s, "solve_ms": st["solve_ms"], "rounds": int(st["rounds"]),
        "pair_evals": int(st["pair_evals"]), "edge_relax": int(st["edge_relax"]),
        "edge_relax_per_s": st["edge_relax"] / (st["solve_ms"] * 1e-3), "roofline": rl,
        "gpu_residual_states": int(res), "oracle_sample_states": int(xs.size), "oracle_sample_mismatches": bad,
        "oracle_first_mismatches": [int(v) for v in first], "oracle_check_s": check_s,
        "finite_fraction": float(fin.mean()), "V_min": int(Vh[fin].min()) if fin.any() else None,
        "V_max_finite": int(Vh[fin].max()) if fin.any() else None,
    }


def aircraft_mission(dims, cone=0, steps=4, samples=2000, timed_solve=True, log=None):
    """The aircraft mission of the paper's example on the device-built
    abstraction (gbf_load_aircraft): problem 1 (back to the runway), then
    problem 2 (over the fire, G_2 = V_1), each loaded (enclosure table, cell
    sets, reverse rows), solved once with per-launch events (roofline) and,
    if timed_solve, once more for the solve time; the GPU's fixed-point
    residual over every state, and the oracle's own check at sampled states
    (its table and sets, one application of the operator)."""
    import numpy as np
    import torch

    import oracle.aircraft as OA
    import paper_2001_06231_amd as gbf
    import synth.aircraft as SA

    log = log or (lambda msg: None)
    dims = tuple(int(v) for v in dims)
    area = (SA.PAPER_AREA[0] * dims[0] // SA.PAPER_DIMS[0], SA.PAPER_AREA[1] * dims[1] // SA.PAPER_DIMS[1])
    sets = "the paper's sets" if not cone and dims == SA.PAPER_DIMS else \
        (f"landing within {cone} degrees at any speed" if cone else "sets scaled with the area")
    out = {"workload": f"aircraft mission (problem 1, then problem 2 with G_2 = V_1) on a "
                       f"{'x'.join(map(str, dims))} grid over {area[0]} m x {area[1]} m, 35 inputs, {sets}; "
                       f"abstraction built on the device, images from the enclosure table",
           "dims": list(dims), "area_m": list(area), "landing_cone_deg": cone or None, "steps_per_period": steps}
    rng = np.random.default_rng(11)
    G_dev = None
    V_prev_host = None
    policies, values, scns = {}, {}, {}
    for stage in (1, 2):
        scn = SA.scenario(dims, area, stage=stage, cone=cone, steps=steps)
        n, K = scn.n, scn.K
        t0 = time.time()
        gr = gbf.load_aircraft(scn, G=G_dev)
        torch.cuda.synchronize()
        load_s = time.time() - t0
        log(f"problem {stage}: loaded n={n} pairs={n * K} in {load_s:.2f}s")
        V = torch.empty(n, dtype=torch.float32, device="cuda")
        status, st_prof, _ = gr.solve(V, profile=True)
        log(f"problem {stage}: profiled solve {st_prof['solve_ms']:.0f} ms, {st_prof['rounds']} rounds")
        st = st_prof
        if timed_solve:
            status, st, _ = gr.solve(V)
            log(f"problem {stage}: solve {st['solve_ms']:.0f} ms")
        pol = torch.empty(n, dtype=torch.int32, device="cuda")
        _, res = gr.policy(pol)
        rl = roofline([st_prof], n * K, PER_EDGE_BYTES["box"])
        rl["kernel"] = "k_ac_relax+k_ac_expand"
        if stage == 1 and dims == SA.PAPER_DIMS and not cone and steps == 4:
            # raw counters (the copy's calibration factor does not carry over
            # to these scattered accesses); per relax step
            rl["traffic"] = read_ac_traffic()
        Vh = V.cpu().numpy()
        t0 = time.time()
        T = OA.table(scn)
        avoid = OA.cell_set(scn, scn.avoid, False)
        reward = OA.cell_set(scn, scn.reward, True) if stage == 2 else np.zeros(1, dtype=bool)
        Gh = (np.where(OA.cell_set(scn, scn.target, True), np.float32(0), np.float32(np.inf)).astype(np.float32)
              if stage == 1 else V_prev_host)
        fin = np.nonzero(np.isfinite(Vh))[0]
        xs = np.concatenate([rng.integers(0, n, samples // 2),
                             fin[rng.integers(0, fin.size, samples // 2)] if fin.size else []])
        bad = OA.sampled_residual(scn, T, Vh, Gh, avoid, reward, xs.astype(np.int64))
        check_s = time.time() - t0
        log(f"problem {stage}: oracle check at {xs.size} states: {bad} mismatches in {check_s:.1f}s")
        out[f"problem{stage}"] = {
            "status": int(status), "enc_used": int(st["enc_used"]), "device_bytes": int(st["device_bytes"]),
            "load_s": load_s, "solve_ms": st["solve_ms"], "rounds": int(st["rounds"]),
            "pair_evals": int(st["pair_evals"]), "edge_relax": int(st["edge_relax"]),
            "expansions": int(st["expansions"]), "marks": int(st["marks"]),
            "edge_relax_per_s": st["edge_relax"] / (st["solve_ms"] * 1e-3), "roofline": rl,
            "gpu_residual_states": int(res), "oracle_sample_states": int(xs.size),
            "oracle_sample_mismatches": int(bad), "oracle_check_s": check_s,
            "finite_states": int(fin.size), "V_max_finite": float(Vh[fin].max()) if fin.size else None,
            "V_min": float(Vh[fin].min()) if fin.size else None}
        if stage == 2:
            out["problem2"]["states_improved_by_reward"] = int((Vh < V_prev_host).sum())
        policies[stage] = pol.cpu().numpy()
        values[stage] = Vh
        scns[stage] = scn
        gr.free()
        G_dev = V
        V_prev_host = Vh
    del G_dev
    torch.cuda.empty_cache()
    out["closed_loop"] = closed_loop(scns, values, policies, rng)
    log(f"closed loop: {out['closed_loop']}")
    return out


def closed_loop(scns, values, policies, rng, start=(840.0, 140.0, 0.0, 53.0)):
    """The mission flown on the real aircraft: its ODE integrated by scipy
    (DOP853) for tau per step, the input chosen by the controller of the cell
    the state is in, held for the step; problem 2's controller until it
    hands over (V2 = G2 = V1 there), then problem 1's until the runway.
    Starts from the paper's start point (840 m, 140 m, heading 0, 53 m/s)
    if the reward lowers its value (V2 < V1 there), else from the centre of
    a random cell where it does (at the start point itself, inside the
    runway-landing set, V2 = V1 = 0 for these seeded fires: the detour does
    not pay).
    Reports the path and whether it stayed safe, reached the runway, and
    spent at most V2 of its start (the method's guarantee)."""
    import math

    import numpy as np
    from scipy.integrate import solve_ivp

    import oracle.aircraft as OA

    s1, s2 = scns[1], scns[2]
    N1, N2, N3, N4 = s1.dims
    eta = np.array([s1.x_max[0] / N1, s1.x_max[1] / N2, 2 * math.pi / N3, (s1.v_range[1] - s1.v_range[0]) / N4])
    lo = np.array([0.0, 0.0, -math.pi, float(s1.v_range[0])])
    avoid = OA.cell_set(s1, s1.avoid, False)
    target = OA.cell_set(s1, s1.target, True)
    reward = OA.cell_set(s2, s2.reward, True) if s2.reward else np.zeros(s2.n, dtype=bool)

    def cell(st):
        c = np.floor((st - lo) / eta).astype(np.int64)
        if c[0] < 0 or c[1] < 0 or c[3] < 0 or c[0] >= N1 or c[1] >= N2 or c[3] >= N4:
            return -1
        return int(c[0] + N1 * (c[1] + N2 * (c[2] % N3 + N3 * c[3])))

    st = np.array([start[0], start[1], math.radians(start[2]), start[3]])
    x0 = cell(st)
    from_paper = x0 >= 0 and bool(values[2][x0] < values[1][x0])
    if not from_paper:
        fin = np.nonzero(values[2] < values[1])[0]
        if fin.size == 0:  # the reward pays nowhere: any controllable cell off the runway
            fin = np.nonzero(np.isfinite(values[2]) & ~target)[0]
        x0 = int(fin[rng.integers(0, fin.size)])
        c = np.array([x0 % N1, (x0 // N1) % N2, (x0 // (N1 * N2)) % N3, x0 // (N1 * N2 * N3)])
        st = lo + (c + 0.5) * eta
    res = {"start": [round(float(v), 3) for v in st], "start_from_paper_point": bool(from_paper),
           "V2_start": float(values[2][x0]), "V1_start": float(values[1][x0])}
    cost, steps, stage, safe, handover, fire_steps = 0.0, [0, 0], 2, True, None, 0
    gus = {k: OA.pair_cost(scns[k]) for k in (1, 2)}
    for _ in range(2000):
        x = cell(st)
        if x < 0 or avoid[x]:
            safe = False
            break
        u = int(policies[stage][x])
        if u == -1:  # hand over: problem 2 to problem 1, or problem 1 at the runway
            if stage == 2:
                handover = [round(float(v), 3) for v in st]
                stage = 1
                continue
            break
        if u < 0:
            safe = False
            break
        scn = scns[stage]
        b = OA.bank_rad(scn, u % scn.n_bank)
        u1 = OA.lib().oracle_ac_thrust(u // scn.n_bank, scn.n_thrust, scn.thrust_max)
        g = float(gus[stage][u])

        def f(t, y, u1=u1, b=b, m=scn.mass):
            return [y[3] * math.cos(y[2]), y[3] * math.sin(y[2]), scn.p_L * y[3] * math.sin(b) / m,
                    (u1 - scn.p_D * y[3] ** 2) / m]

        st = solve_ivp(f, (0.0, scn.tau), list(st), method="DOP853", rtol=1e-10, atol=1e-10).y[:, -1]
        st[2] = (st[2] + math.pi) % (2 * math.pi) - math.pi
        if stage == 2:
            y = cell(st)
            cost += float(s2.reward_cost) if (y >= 0 and reward[y]) else g
        else:
            cost += g
        steps[2 - stage] += 1
        if stage == 2 and y >= 0 and reward[y]:
            fire_steps += 1
    x = cell(st)
    res.update({"handover": handover, "end": [round(float(v), 3) for v in st], "steps_problem2": steps[0],
                "steps_problem1": steps[1], "steps_in_fire": fire_steps, "cost": round(cost, 4), "safe": bool(safe),
                "reached_runway": bool(x >= 0 and target[x]),
                "cost_within_V2": bool(cost <= res["V2_start"] + 1e-3)})
    return res


def aircraft_run(args):
    """--aircraft: the mission on the grid given; prints one JSON object."""
    def log(msg):
        print(f"[aircraft] {msg}", file=sys.stderr, flush=True)

    import torch
    torch.cuda.set_device(0)
    if args.calib_copy:
        # a plain 256 MiB device copy: reference for the HBM byte counters
        x = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    return aircraft_mission(args.aircraft_grid.split("x"), args.aircraft_cone, args.aircraft_steps,
                            args.aircraft_samples, log=log)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="auto", choices=["persistent", "hostloop", "single_block", "auto"])
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy", action="store_true", help="run a 256 MiB device copy first (counter reference)")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the main workload (no other configs, batch or learned comparison)")
    ap.add_argument("--learned-eval", type=int, default=0,
                    help="instead: evaluate the trained network on this many held-out instances")
    ap.add_argument("--eval-reps", type=int, default=3)
    ap.add_argument("--paper-scale", action="store_true",
                    help="instead: the 141.75 M-cell, 35-input grid with 64-bit pair ids (~200 GB of device memory)")
    ap.add_argument("--paper-expand", type=int, default=2, help="expand_box for --paper-scale (2 = reverse CSR)")
    ap.add_argument("--paper-samples", type=int, default=1000000)
    ap.add_argument("--aircraft", action="store_true",
                    help="instead: the aircraft mission on the device-built abstraction")
    ap.add_argument("--aircraft-grid", default="200x70x75x135",
                    help="cells on x1, x2, heading, speed (the area scales with the first two)")
    ap.add_argument("--aircraft-samples", type=int, default=2000)
    ap.add_argument("--no-aircraft", action="store_true",
                    help="leave the aircraft mission on the paper's grid out of the default run")
    ap.add_argument("--aircraft-cone", type=int, default=0,
                    help="landing headings within +-cone degrees at any speed (0 = the paper's landing set)")
    ap.add_argument("--aircraft-steps", type=int, default=4, help="integration steps per sampling period")
    ap.add_argument("--workers", type=int, default=8,
                    help="worker processes for input generation and the CPU oracle (1 = none, e.g. under a "
                         "profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the solver has no multi-GPU "
              "path", file=sys.stderr)
        sys.exit(2)
    # the worker processes are forked before the first GPU call
    pool = None
    if args.workers > 1 and not args.paper_scale and not args.aircraft and (
            args.learned_eval or not args.no_extras or not args.no_cpu):
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(args.workers)
    try:
        if args.paper_scale:
            print(json.dumps(paper_scale_run(args)), flush=True)
        elif args.aircraft:
            print(json.dumps(aircraft_run(args)), flush=True)
        elif args.learned_eval:
            print(json.dumps(learned_eval(args, pool)), flush=True)
        else:
            print(json.dumps(run(args, pool)), flush=True)
    finally:
        if pool is not None:
            pool.terminate()


if __name__ == "__main__":
    main()
