"""Training and use of the frontier-ordering network.

The network (gbf_mlp_* in include/gbf.h) is trained on value functions that
the solver itself produced on instances of one family (here: the 4-D grids
60x60x30x12 with 16 inputs, random target and obstacle placements), then
gives every state of a new instance a bucket key for the bucket-ordered
solve.  Every arithmetic step (features, forward, backward, Adam, keys)
runs in the library's kernels; this module draws the random numbers (weight
initialisation, sample cells, minibatch order) from the seeded streams of
`synth` and passes them in.

Command line (writes the trained weights as text):
    python -m paper_2001_06231_amd.learn --train 256 --out <file>
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

from . import MLP, MLP_NPARAMS, load_problem

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "mlp_grid4d_60x60x30x12_k16.txt")
SCALE = 1000.0   # the network predicts V / SCALE
WIDTH = 16.0     # bucket width in V units


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    import synth
    s = synth.Stream(seed, 0x4D4C50)
    p = np.zeros(MLP_NPARAMS, np.float64)
    u = s.uniform(MLP_NPARAMS) * 2.0 - 1.0
    p[0:256] = u[0:256] * np.sqrt(6.0 / 4)         # W1
    p[320:4416] = u[320:4416] * np.sqrt(6.0 / 64)  # W2
    p[4480:4544] = u[4480:4544] * np.sqrt(6.0 / 64)  # W3
    return p.astype(np.float32)


def target_centre(prob):
    """Centre (in cell units, axes 0 and 1) of the states with finite G."""
    from . import INF_I32
    G = np.asarray(prob.G)
    fin = G != INF_I32 if G.dtype == np.int32 else np.isfinite(G)
    cells = np.nonzero(fin)[0]
    if cells.size == 0:
        return 0.0, 0.0
    N0, N1 = int(prob.dims[0]), int(prob.dims[1])
    return float((cells % N0 + 0.5).mean()), float(((cells // N0) % N1 + 0.5).mean())


def save_params(params, path, meta=""):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("# frontier-ordering network 4-64-64-1, fp32 master weights, one per line\n")
        for line in meta.strip().splitlines():
            f.write(f"# {line}\n")
        for v in np.asarray(params, np.float32):
            f.write(f"{float(v).hex()}\n")


def load_params(path=WEIGHTS) -> np.ndarray:
    vals = [float.fromhex(line.strip()) for line in open(path) if line.strip() and not line.startswith("#")]
    p = np.array(vals, dtype=np.float32)
    if p.shape != (MLP_NPARAMS,):
        raise ValueError(f"{path}: expected {MLP_NPARAMS} parameters, found {p.size}")
    return p


def _gen(index):
    import synth
    return synth.learned_instance(index, with_csr=False)


def make_pool(workers):
    """Generator worker processes (plain numpy).  Create the pool before the
    first GPU call of the process: the workers are forked from it."""
    if workers <= 1:
        return None
    import multiprocessing as mp
    return mp.get_context("fork").Pool(workers)


def instances(indices, pool=None):
    """Yields (index, problem) in order, generated in `pool` if given."""
    if pool is None:
        for i in indices:
            yield i, _gen(i)
        return
    for i, p in zip(indices, pool.imap(_gen, indices)):
        yield i, p


class SampleSet:
    """Device-resident (features, labels) gathered from solved instances."""

    def __init__(self, net, capacity):
        import torch
        self.net = net
        self.feat = torch.empty((capacity, 4), dtype=torch.float32, device="cuda")
        self.target = torch.empty(capacity, dtype=torch.float32, device="cuda")
        self.size = 0

    def add(self, prob, V, cells):
        """V: device values of a solved instance; cells: device int64."""
        cnt = int(cells.numel())
        f, t = self.net.samples(prob.dims, target_centre(prob), cells, V=V, scale=SCALE)
        self.feat[self.size:self.size + cnt].copy_(f)
        self.target[self.size:self.size + cnt].copy_(t)
        self.size += cnt


def solve_plain(prob, stream=None):
    import torch
    g = load_problem(prob, encoding="csr", stream=stream)
    V = torch.empty(prob.n, dtype=torch.int32, device="cuda")
    st, stats, _ = g.solve(V)
    return g, V, stats


def train(net, data, epochs, batch, lr, seed, log=None):
    """Minibatch Adam over the sample set; the order of each epoch is a
    permutation drawn from synth's stream.  Returns the mean loss per epoch."""
    import torch
    import synth
    s = synth.Stream(seed, 0x7E4)
    n = data.size
    feat, target = data.feat[:n], data.target[:n]
    losses = []
    for ep in range(epochs):
        perm = np.argsort(s.raw(n))
        idx = torch.from_numpy(perm.astype(np.int64)).cuda()
        tot, cnt = 0.0, 0
        for b0 in range(0, n, batch):
            want = (b0 // batch) % 64 == 0
            loss = net.train_step(feat, target, idx[b0:b0 + batch], lr=lr, want_loss=want)
            if want:
                tot += loss
                cnt += 1
        losses.append(tot / max(1, cnt))
        if log:
            log(f"epoch {ep}: sampled minibatch loss {losses[-1]:.5f}")
    return losses


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=256, help="training instances (indices 0..N-1)")
    ap.add_argument("--samples", type=int, default=32768, help="sample cells per instance")
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--out", default=WEIGHTS)
    a = ap.parse_args(argv)
    pool = make_pool(a.workers)
    import torch
    import synth
    torch.cuda.set_device(0)
    t0 = time.time()

    def log(msg):
        print(f"[learn {time.time() - t0:7.1f}s] {msg}", flush=True)

    net = MLP(init_params(a.seed))
    data = SampleSet(net, a.train * a.samples)
    for i, prob in instances(list(range(a.train)), pool):
        g, V, st = solve_plain(prob)
        cs = synth.Stream(synth.instance_seed(5, i), 0x5A)
        cells = torch.from_numpy((cs.raw(a.samples) % np.uint64(prob.n)).astype(np.int64)).cuda()
        data.add(prob, V, cells)
        g.free()
        log(f"instance {i}: solved in {st['solve_ms']:.1f} ms, {data.size} samples")
    if pool is not None:
        pool.close()
        pool.join()
    losses = train(net, data, a.epochs, a.batch, a.lr, a.seed, log)
    master, _ = net.params()
    save_params(master, a.out, meta=(f"trained on instances 0..{a.train - 1} of the 60x60x30x12 K=16 int32 family, "
                                     f"{a.samples} sample cells each, {a.epochs} epochs, batch {a.batch}, "
                                     f"lr {a.lr}, seed {a.seed}\nsampled minibatch loss per epoch: "
                                     + " ".join(f"{v:.5f}" for v in losses)))
    log(f"wrote {a.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
