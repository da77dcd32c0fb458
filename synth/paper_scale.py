"""The paper-scale synthetic grid: 200 x 70 x 75 x 135 = 141.75 M cells and 35
inputs, the size of the auxiliary problems of the firefighting example
(Sect. VI-A: the state space subdivided into 200*70*75*135 hyper-rectangles,
35 abstract inputs), about 4.96 G (x,u) pairs.

Like the other grid workloads it is a synthetic stand-in (the paper's
abstraction needs the aircraft's attainable sets and scenario sets that are
not available): axes (x, y, heading, speed); each input has a fixed drift
(35 = 5 thrust levels x 7 bank levels, the vertices of the paper's 4 x 6
subdivision of the input range): the bank level sets the heading drift, the
thrust level the speed drift, and the input index one of 8 planar
directions.  F(x,u) is the box [x+d, x+d+e] per axis (spread in the drift
direction), e in {0,1} with P(1) = 0.3 per axis, clamped to the grid.  The
running cost is in potential form with a separable potential
phi(x) = p0(x0) + p1(x1) + p2(x2) + p3(x3) (four smoothed random integer
profiles in [0,100]):

    g(x,u) = c(x,u) + phi(x) - min_{y in F(x,u)} phi(y),  c in U{1..8},

so costs take both signs and no negative cycle exists.  The target is a
6 x 6 planar slab over all headings and speeds; obstacles are planar
blocks over all headings and speeds covering >= 5% of the plane.

Every per-pair quantity is a function of the pair id through the
counter-based SplitMix64 of `synth`, so the arrays can be built in chunks
on the device (torch integer ops, 60 GB) and any sampled row recomputed on
the host, identically, for the oracle's check.  Nothing here is solver
arithmetic.
"""
from __future__ import annotations

import numpy as np

from . import INF_I32, Stream, _gauss_kernel, _mix64, instance_seed

DIMS = (200, 70, 75, 135)
K = 35
P_EXT = 77  # extent 1 when a hash byte is below this: 77/256 = 0.30

_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_GOLDEN = 0x9E3779B97F4A7C15


def _s64(v: int) -> int:
    """A 64-bit pattern as the signed value torch's int64 holds."""
    v &= 0xFFFFFFFFFFFFFFFF
    return v - (1 << 64) if v >= (1 << 63) else v


def _srl(z, k: int):
    """Logical right shift of int64 tensors (torch's >> is arithmetic)."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def mix64_torch(z):
    """SplitMix64's finaliser on int64 tensors (wrapping arithmetic); the
    same function as synth._mix64 on uint64 arrays."""
    z = z ^ _srl(z, 30)
    z = z * _s64(_M1)
    z = z ^ _srl(z, 27)
    z = z * _s64(_M2)
    return z ^ _srl(z, 31)


def drifts() -> np.ndarray:
    """[35, 4] drift per input: input u = 7*thrust + bank (thrust 0..4, bank
    0..6); heading drift sign(bank - 3), speed drift clip(thrust - 2, -1, 1),
    planar drift the compass direction u mod 8."""
    compass = [(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1)]
    out = np.zeros((K, 4), dtype=np.int64)
    for t in range(5):
        for b in range(7):
            u = 7 * t + b
            out[u, 0], out[u, 1] = compass[u % 8]
            out[u, 2] = int(np.sign(b - 3))
            out[u, 3] = int(np.clip(t - 2, -1, 1))
    return out


def meta(seed: int | None = None) -> dict:
    """Everything that is not per pair: the potential profiles, drifts,
    target rectangle, obstacle footprint and the hash state."""
    s = instance_seed(6, 0) if seed is None else seed
    prof = []
    for a, N in enumerate(DIMS):
        r = Stream(s, 10 + a)
        f = r.integers(0, (1 << 20) - 1, N).astype(np.float64)
        w = _gauss_kernel(max(1.0, N / 10.0))
        rr = (w.size - 1) // 2
        p = np.pad(f, (rr, rr), mode="reflect" if N > rr else "symmetric")
        f = np.convolve(p, w, mode="valid")
        f = (f - f.min()) / max(f.max() - f.min(), 1e-300) * 100.0
        prof.append(np.rint(f).astype(np.int64))
    rt = Stream(s, 2)
    t0 = int(rt.integers(0, DIMS[0] - 6, 1)[0])
    t1 = int(rt.integers(0, DIMS[1] - 6, 1)[0])
    ra = Stream(s, 3)
    foot = np.zeros((DIMS[1], DIMS[0]), dtype=bool)  # [x1, x0]
    tfoot = np.zeros_like(foot)
    tfoot[t1:t1 + 6, t0:t0 + 6] = True
    while foot.sum() < 0.05 * DIMS[0] * DIMS[1]:
        w = int(ra.integers(3, 12, 1)[0])
        h = int(ra.integers(3, 8, 1)[0])
        a0 = int(ra.integers(0, DIMS[0] - w, 1)[0])
        a1 = int(ra.integers(0, DIMS[1] - h, 1)[0])
        blk = np.zeros_like(foot)
        blk[a1:a1 + h, a0:a0 + w] = True
        if (blk & tfoot).any():
            continue
        foot |= blk
    state = int(_mix64(np.array([np.uint64((s ^ 0x5EED0001) & 0xFFFFFFFFFFFFFFFF)], dtype=np.uint64))[0])
    return {"seed": s, "profiles": prof, "drift": drifts(), "target": (t0, t1), "foot": foot, "state": state,
            "n": int(np.prod(DIMS)), "K": K, "dims": DIMS}


def pair_rows(pids, m: dict):
    """Packed box (int64 tensor holding the uint64 pattern) and int32 cost of
    the pairs `pids` (int64 tensor, any device)."""
    import torch
    dev = pids.device
    N = torch.tensor(DIMS, dtype=torch.int64, device=dev)
    st = torch.tensor([1, DIMS[0], DIMS[0] * DIMS[1], DIMS[0] * DIMS[1] * DIMS[2]], dtype=torch.int64, device=dev)
    drift = torch.as_tensor(m["drift"], dtype=torch.int64, device=dev)
    x = pids // K
    u = pids - x * K
    h = mix64_torch((pids + 1) * _s64(_GOLDEN) + _s64(m["state"]))
    coords = [(x // st[a]) % N[a] for a in range(4)]
    lo_lin = torch.zeros_like(pids)
    hi_pack = torch.zeros_like(pids)
    phi_x = torch.zeros_like(pids)
    phi_min = torch.zeros_like(pids)
    for a in range(4):
        pa = torch.as_tensor(m["profiles"][a], dtype=torch.int64, device=dev)
        e = (_srl(h, 8 * a) & 0xFF) < P_EXT
        e = e.to(torch.int64)
        d = drift[u, a]
        shift = torch.where(d < 0, d - e, d)
        lo = torch.clamp(coords[a] + shift, 0, DIMS[a] - 1)
        hi = torch.clamp(coords[a] + shift + e, 0, DIMS[a] - 1)
        lo_lin += lo * st[a]
        hi_pack |= (hi - lo) << (8 * a)
        phi_x += pa[coords[a]]
        phi_min += torch.minimum(pa[lo], pa[hi])
    c = 1 + ((_srl(h, 32) * 8) >> 32)
    g = (c + phi_x - phi_min).to(torch.int32)
    box = lo_lin | (hi_pack << 32)
    return box, g


def state_rows(xs, m: dict):
    """Terminal cost (int32) and avoid flag (uint8) of the states `xs`."""
    import torch
    dev = xs.device
    x0 = xs % DIMS[0]
    x1 = (xs // DIMS[0]) % DIMS[1]
    t0, t1 = m["target"]
    tgt = (x0 >= t0) & (x0 < t0 + 6) & (x1 >= t1) & (x1 < t1 + 6)
    G = torch.where(tgt, torch.zeros_like(xs), torch.full_like(xs, int(INF_I32))).to(torch.int32)
    foot = torch.as_tensor(m["foot"].reshape(-1), dtype=torch.uint8, device=dev)
    av = foot[x1 * DIMS[0] + x0]
    return G, av


def build(m: dict, device="cuda", chunk=1 << 25, log=None):
    """Full arrays on `device`: box (int64 [n*K], uint64 pattern), g (int32
    [n*K]), G (int32 [n]), avoid (uint8 [n]), generated chunk by chunk."""
    import torch
    n = m["n"]
    npairs = n * K
    box = torch.empty(npairs, dtype=torch.int64, device=device)
    g = torch.empty(npairs, dtype=torch.int32, device=device)
    for p0 in range(0, npairs, chunk):
        p1 = min(npairs, p0 + chunk)
        b, c = pair_rows(torch.arange(p0, p1, dtype=torch.int64, device=device), m)
        box[p0:p1] = b
        g[p0:p1] = c
        if log and (p0 // chunk) % 32 == 0:
            log(f"pairs {p1}/{npairs}")
    G = torch.empty(n, dtype=torch.int32, device=device)
    av = torch.empty(n, dtype=torch.uint8, device=device)
    for x0 in range(0, n, chunk):
        x1 = min(n, x0 + chunk)
        a, b = state_rows(torch.arange(x0, x1, dtype=torch.int64, device=device), m)
        G[x0:x1] = a
        av[x0:x1] = b
    return box, g, G, av


def sample_states(count: int, m: dict, seed: int = 99) -> np.ndarray:
    """`count` distinct uniformly drawn states (ascending)."""
    r = Stream(m["seed"], 1000 + seed)
    xs = np.unique(r.integers(0, m["n"] - 1, int(count * 1.05) + 16))
    return xs[:count] if xs.size >= count else xs
