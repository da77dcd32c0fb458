"""Host logic of bench.py (no GPU): the algorithmic-bytes model behind the
roofline, the committed traffic summary it reads, and the one-GPU guard."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_model():
    st = {"pair_evals": 10, "edge_relax": 180, "expansions": 3, "marks": 600}
    # relax: 20 per pair + 8 per edge; expansion: 8 per state + 5 per mark
    assert bench.algorithmic_bytes(st, 1000, "hostloop", 7) == 20 * 10 + 8 * 180 + 8 * 3 + 5 * 600
    # the persistent and single-block kernels also read the map once per round
    # (rounds + 1 scans) and write 4 bytes per listed pair
    want = 20 * 10 + 8 * 180 + 8 * 3 + 5 * 600 + 8 * 1000 + 4 * 10
    assert bench.algorithmic_bytes(st, 1000, "persistent", 7) == want
    assert bench.algorithmic_bytes(st, 1000, "single_block", 7) == want


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
