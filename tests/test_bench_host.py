"""Host logic of bench.py (no GPU): the algorithmic-bytes model behind the
roofline, the committed traffic summary it reads, and the one-GPU guard."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_model():
    st = {"pair_evals": 10, "edge_relax": 180, "expansions": 3, "marks": 600, "rounds": 7}
    # relax: 20 per pair + 8 per CSR successor; expansion: 8 per state + 8 per
    # visited predecessor pair
    base = 20 * 10 + 8 * 3 + 8 * 600
    assert bench.algorithmic_bytes(st, 1000, 8, "hostloop") == base + 8 * 180
    # box successors: 4 bytes per successor (no index stream)
    assert bench.algorithmic_bytes(st, 1000, 4, "hostloop") == base + 4 * 180
    # the persistent and single-block kernels also read and clear the
    # frontier once per round (rounds + 1 scans of nK/4 bytes) and write 4
    # bytes per listed pair
    want = base + 8 * 180 + 8 * 1000 / 4 + 4 * 10
    assert bench.algorithmic_bytes(st, 1000, 8, "persistent") == want
    assert bench.algorithmic_bytes(st, 1000, 8, "single_block") == want


def test_roofline_from_profiled_solves():
    """achieved = algorithmic bytes per launch over the average launch time."""
    import paper_2001_06231_amd as gbf
    st = {"pair_evals": 1000, "edge_relax": 16000, "expansions": 100, "marks": 20000, "rounds": 5,
          "relax_launches": 10, "relax_ms": 0.5, "mode_used": gbf.MODE_HOSTLOOP}
    r = bench.roofline([st, st], 4096, 8)
    per_launch = (20 * 1000 + 8 * 16000 + 8 * 100 + 8 * 20000) / 10
    assert r["kernel"] == "k_relax" and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert abs(r["algorithmic_bytes_per_launch"] - per_launch) < 1e-6
    assert abs(r["achieved"] - per_launch / 0.05e-3 / 1e9) < 1e-6
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12


def test_cpu_job_pins_one_core():
    """The CPU baseline runs the oracle in a process pinned to one core."""
    import os as _os
    core = sorted(_os.sched_getaffinity(0))[-1]
    before = _os.sched_getaffinity(0)
    label, r = bench.cpu_job(("t", ["grid2d"], 1, None, core))
    assert _os.sched_getaffinity(0) == {core}
    _os.sched_setaffinity(0, before)
    assert r["cores"] == 1 and r["pinned_core"] == core and r["value"] > 0 and r["edge_relax"] > 0


def test_traffic_read_only_for_the_same_kernel_source(tmp_path, monkeypatch):
    """A counter summary is used only for the kernel and the kernel source
    it was taken on."""
    f = tmp_path / "traffic.txt"
    f.write_text(f"# header\nkernel: k_relax\nkernel_source_sha256_16: {bench.kernel_source_hash()}\n"
                 "hbm_bytes_per_launch: 1234.0\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.read_traffic("k_relax") == 1234.0
    assert bench.read_traffic("k_persistent") is None
    f.write_text("kernel: k_relax\nkernel_source_sha256_16: 0000000000000000\nhbm_bytes_per_launch: 1.0\n")
    assert bench.read_traffic("k_relax") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.read_traffic("k_relax") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)


def test_cpu_job_reward_chain(monkeypatch):
    """The reward chain's CPU baseline times only the second problem, whose
    terminal cost is the oracle's value function of the first."""
    import numpy as np

    import oracle
    import synth
    small = synth.grid4d(synth.instance_seed(2, 41), dims=(10, 9, 6, 4))
    monkeypatch.setattr(bench, "make_problem", lambda kind: small)
    label, r = bench.cpu_job(("reward", ["reward:grid4d_i32"], 1, None, None))
    p2 = synth.reward_problem(small, oracle.solve(small)["V"], bench.REWARD_SEED)
    want = oracle.solve(p2)["counters"]["edge_relax"]
    assert label == "reward" and r["edge_relax"] == want and r["value"] > 0
    assert np.array_equal(p2.G, oracle.solve(small)["V"])


def test_closed_loop_flight_on_the_oracle_controller():
    """bench.closed_loop flies the mission on the ODE with given controllers:
    with the oracle's, every flight (from a cell where the reward lowers the
    value, else from any controllable cell) stays safe, reaches the runway
    and keeps within V2."""
    import numpy as np

    import oracle
    import oracle.aircraft as OA
    import synth.aircraft as SA
    s1, s2 = SA.small(1), SA.small(2)
    r1 = oracle.solve(OA.problem(s1), precision="f32")
    r2 = oracle.solve(OA.problem(s2, G=r1["V"]), precision="f32")
    for seed in range(3):
        res = bench.closed_loop({1: s1, 2: s2}, {1: r1["V"], 2: r2["V"]}, {1: r1["policy"], 2: r2["policy"]},
                                np.random.default_rng(seed))
        assert res["safe"] and res["reached_runway"] and res["cost_within_V2"], res
        assert res["V2_start"] <= res["V1_start"]
