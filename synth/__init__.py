"""Seeded synthetic problem instances for the generalized Bellman-Ford solver.

This module only *builds inputs*: optimal control problems (X, U, F, G, g) in
the sense of the paper's Definition of an optimal control problem (Sect. III-C).
It contains none of the solver's arithmetic (no dynamic-programming operator,
no frontier, no value function).  Both the CPU oracle and the HIP library are
fed from here; nothing here depends on either of them.

Instances are regular grids of hyper-rectangular cells, the cover that the
paper uses for its discrete abstractions (Sect. V-B), with box-shaped
successor sets F(x,u) as produced by rectangular over-approximations of
attainable sets (Sect. V-B).  Costs follow a "potential form"

    g(x,u) = c(x,u) + phi(x) - min_{y in F(x,u)} phi(y),   c >= c_min > 0,

so g takes both signs (the paper's reward mechanism of Sect. VI-A needs
negative running costs) while every cycle has positive total cost, hence no
negative cycles exist (sum of g along a cycle >= cycle length * c_min).

Random numbers come from a project-written SplitMix64 (Steele, Lea, Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014), counter based
so that any element of any stream can be drawn independently.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

INF_I32 = np.int32(2**31 - 1)
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_ROOT_SEED = 0x200106231


# --------------------------------------------------------------------------
# SplitMix64, vectorised.  output_i = mix(state0 + (i+1) * golden)
# --------------------------------------------------------------------------
def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def _u64(v: int) -> np.uint64:
    return np.uint64(v & 0xFFFFFFFFFFFFFFFF)


class Stream:
    """A counter-based SplitMix64 stream; draws are consumed sequentially."""

    def __init__(self, seed: int, tag: int):
        base = np.array([_u64(seed) ^ _u64(tag * 0xD1B54A32D192ED03)], dtype=np.uint64)
        self._state = _mix64(base)[0]
        self._ctr = 0

    def raw(self, size: int) -> np.ndarray:
        idx = np.arange(self._ctr + 1, self._ctr + 1 + size, dtype=np.uint64)
        self._ctr += size
        with np.errstate(over="ignore"):
            z = idx * _GOLDEN + self._state
        return _mix64(z)

    def integers(self, lo: int, hi: int, size: int) -> np.ndarray:
        """Uniform integers in [lo, hi] (inclusive), multiply-shift on 32 bits."""
        span = np.uint64(hi - lo + 1)
        top = self.raw(size) >> np.uint64(32)
        return (lo + ((top * span) >> np.uint64(32)).astype(np.int64)).astype(np.int64)

    def uniform(self, size: int) -> np.ndarray:
        """Uniform doubles in [0, 1) with 53 random bits."""
        return (self.raw(size) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)

    def choice_p(self, probs: Sequence[float], size: int) -> np.ndarray:
        """Categorical draw over range(len(probs))."""
        u = self.uniform(size)
        cdf = np.cumsum(np.asarray(probs, dtype=np.float64))
        cdf[-1] = 1.0
        return np.searchsorted(cdf, u, side="right").astype(np.int64)


def instance_seed(config: int, index: int) -> int:
    """Seed of instance `index` of workload `config`."""
    x = np.array([_u64(_ROOT_SEED ^ (config << 32) ^ index)], dtype=np.uint64)
    return int(_mix64(x)[0])


# --------------------------------------------------------------------------
# Problem container
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """An optimal control problem (X, U, F, G, g) on a grid.

    States are linear cell indices x = x0 + N0*(x1 + N1*(x2 + N2*x3)); the
    pair (x,u) has id p = x*K + u.  F(x,u) is the box of cells
    [lo, lo+ext] (per axis, inclusive).  `succ_ptr/succ_idx` is the same
    relation as CSR with each row listed in ascending cell order.
    `g` is per pair (int32 or float32), `G` per state; INF means "not a
    target" / "forbidden input".  `avoid` cells are states the controller
    must never enter.
    """
    dims: tuple            # 4 entries, padded with 1
    ndim: int
    K: int
    dtype: str             # "i32" or "f32"
    G: np.ndarray          # [n]
    g: np.ndarray          # [n*K]
    avoid: np.ndarray      # [n] uint8
    box_lo: Optional[np.ndarray] = None   # [n*K] uint32 linear low corner
    box_ext: Optional[np.ndarray] = None  # [n*K, 4] uint8
    succ_ptr: Optional[np.ndarray] = None  # [n*K+1] int64 (fits int32 for all workloads)
    succ_idx: Optional[np.ndarray] = None  # [m] int32
    target: Optional[np.ndarray] = None   # [n] bool
    phi: Optional[np.ndarray] = None      # [n] potential used to build g
    cost_c: Optional[np.ndarray] = None   # [n*K] positive part of g
    c_min: float = 0.0
    name: str = ""
    g_edge: Optional[np.ndarray] = None   # [m] per-edge part h of the running cost
                                          # g(x,y,u) = g(x,u) + h(x,y,u), CSR order

    @property
    def n(self) -> int:
        return int(self.G.shape[0])

    @property
    def npairs(self) -> int:
        return self.n * self.K

    @property
    def m(self) -> int:
        return int(self.succ_ptr[-1]) if self.succ_ptr is not None else int(self.box_sizes().sum())

    def box_packed(self) -> np.ndarray:
        """8 bytes per pair: low 32 bits = low-corner cell, high 32 bits =
        ext0 | ext1<<8 | ext2<<16 | ext3<<24."""
        e = self.box_ext.astype(np.uint64)
        hi = e[:, 0] | (e[:, 1] << np.uint64(8)) | (e[:, 2] << np.uint64(16)) | (e[:, 3] << np.uint64(24))
        return (self.box_lo.astype(np.uint64) | (hi << np.uint64(32))).astype(np.uint64)

    def box_sizes(self) -> np.ndarray:
        e = self.box_ext.astype(np.int64) + 1
        return e[:, 0] * e[:, 1] * e[:, 2] * e[:, 3]

    def ensure_csr(self) -> "Problem":
        if self.succ_ptr is None:
            self.succ_ptr, self.succ_idx = boxes_to_csr(self.dims, self.box_lo, self.box_ext)
        return self


def strides(dims) -> np.ndarray:
    d = list(dims)
    return np.array([1, d[0], d[0] * d[1], d[0] * d[1] * d[2]], dtype=np.int64)


def cell_coords(dims) -> np.ndarray:
    """[n, 4] int64 coordinates of every cell (axis 0 fastest)."""
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    out = np.empty((n, 4), dtype=np.int64)
    rem = idx
    for a in range(4):
        out[:, a] = rem % dims[a]
        rem = rem // dims[a]
    return out


def _box_shapes(ext: np.ndarray):
    """Shape id of every box and the list of distinct shapes (w0,w1,w2,w3)."""
    e = ext.astype(np.int64)
    emax = e.max(axis=0) + 1 if e.shape[0] else np.ones(4, dtype=np.int64)
    sid = e[:, 0] + emax[0] * (e[:, 1] + emax[1] * (e[:, 2] + emax[2] * e[:, 3]))
    return sid, emax


def boxes_to_csr(dims, lo: np.ndarray, ext: np.ndarray):
    """Expand boxes into ascending CSR rows (generator-side expansion).

    Within a box the cells are listed in ascending linear order, i.e.
    lexicographically in (j3, j2, j1, j0) with offsets j_a in [0, ext_a].
    Pairs are grouped by box shape so that each group is one broadcast."""
    st = strides(dims)
    e = ext.astype(np.int64)
    sizes = (e[:, 0] + 1) * (e[:, 1] + 1) * (e[:, 2] + 1) * (e[:, 3] + 1)
    ptr = np.zeros(lo.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes, out=ptr[1:])
    idx = np.empty(int(ptr[-1]), dtype=np.int32)
    sid, emax = _box_shapes(ext)
    order = np.argsort(sid, kind="stable")
    bounds = np.searchsorted(sid[order], np.arange(int(np.prod(emax)) + 1))
    base = lo.astype(np.int64)
    for shape in range(int(np.prod(emax))):
        sel = order[bounds[shape]:bounds[shape + 1]]
        if sel.size == 0:
            continue
        w0 = shape % emax[0]
        r = shape // emax[0]
        w1 = r % emax[1]
        r //= emax[1]
        w2 = r % emax[2]
        w3 = r // emax[2]
        j3, j2, j1, j0 = np.meshgrid(np.arange(w3 + 1), np.arange(w2 + 1), np.arange(w1 + 1),
                                     np.arange(w0 + 1), indexing="ij")
        offs = (j0 * st[0] + j1 * st[1] + j2 * st[2] + j3 * st[3]).reshape(-1)
        k = offs.size
        pos = ptr[sel][:, None] + np.arange(k)[None, :]
        idx[pos.reshape(-1)] = (base[sel][:, None] + offs[None, :]).reshape(-1).astype(np.int32)
    return ptr, idx


def box_min(dims, lo: np.ndarray, ext: np.ndarray, field: np.ndarray, csr=None) -> np.ndarray:
    """min of `field` over each box (input construction only), by separable
    window minima: for every extent combination the field of minima over
    [x, x+e] per axis is built once, then each box reads its corner."""
    if csr is not None:
        ptr, idx = csr
        return np.minimum.reduceat(field[idx], ptr[:-1].astype(np.intp))
    st = strides(dims)
    f = field.astype(np.float64)
    n = f.size
    e = ext.astype(np.int64)
    emax = e.max(axis=0)

    def window(g, a, w):
        # min over cells x, x+st_a, ..., x+w*st_a (only read where in range)
        out = g.copy()
        for j in range(1, w + 1):
            sh = np.full(n, np.inf)
            sh[:n - j * st[a]] = g[j * st[a]:]
            np.minimum(out, sh, out=out)
        return out

    out = np.empty(lo.shape[0])
    lo64 = lo.astype(np.int64)
    sid, smax = _box_shapes(ext)
    order = np.argsort(sid, kind="stable")
    bounds = np.searchsorted(sid[order], np.arange(int(np.prod(smax)) + 1))
    for e0 in range(emax[0] + 1):
        f0 = window(f, 0, e0)
        for e1 in range(emax[1] + 1):
            f1 = window(f0, 1, e1)
            for e2 in range(emax[2] + 1):
                f2 = window(f1, 2, e2)
                for e3 in range(emax[3] + 1):
                    shape = e0 + smax[0] * (e1 + smax[1] * (e2 + smax[2] * e3))
                    sel = order[bounds[shape]:bounds[shape + 1]]
                    if sel.size == 0:
                        continue
                    f3 = window(f2, 3, e3)
                    out[sel] = f3[lo64[sel]]
    return out


def _gauss_kernel(sigma: float) -> np.ndarray:
    r = max(1, int(math.ceil(3.0 * sigma)))
    k = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return w / w.sum()


def smooth_field(dims, sigmas, rng: Stream, top: float, integer: bool) -> np.ndarray:
    """iid integers in [0, 2^20) per cell -> separable Gaussian blur (fp64,
    mirrored borders) -> min-max rescale to [0, top] -> round half-even if
    `integer`.  Returns a flat [n] array (axis 0 fastest)."""
    n = int(np.prod(dims))
    f = rng.integers(0, (1 << 20) - 1, n).astype(np.float64)
    f = f.reshape(tuple(reversed(dims)))        # C order: last axis = axis 0
    for a in range(4):
        if dims[a] <= 1 or sigmas[a] <= 0:
            continue
        ax = 3 - a
        w = _gauss_kernel(sigmas[a])
        r = (w.size - 1) // 2
        padw = [(0, 0)] * 4
        padw[ax] = (r, r)
        mode = "reflect" if dims[a] > r else "symmetric"
        p = np.pad(f, padw, mode=mode)
        acc = np.zeros_like(f)
        for k in range(w.size):
            sl = [slice(None)] * 4
            sl[ax] = slice(k, k + dims[a])
            acc += w[k] * p[tuple(sl)]
        f = acc
    f = f.reshape(-1)
    lo, hi = f.min(), f.max()
    f = (f - lo) / (hi - lo if hi > lo else 1.0) * top
    if integer:
        return np.rint(f).astype(np.int64)
    return f


# --------------------------------------------------------------------------
# Grid problem builder
# --------------------------------------------------------------------------
def drifts_for(ndim: int, K: int) -> np.ndarray:
    """Fixed drift per input: +-e_i per axis, then (+-1,+-1,0,0), then
    (0,0,+-1,+-1), truncated to K entries."""
    out = []
    for a in range(ndim):
        for s in (+1, -1):
            v = [0, 0, 0, 0]
            v[a] = s
            out.append(v)
    if ndim >= 2:
        for s0 in (+1, -1):
            for s1 in (+1, -1):
                out.append([s0, s1, 0, 0])
    if ndim >= 4:
        for s2 in (+1, -1):
            for s3 in (+1, -1):
                out.append([0, 0, s2, s3])
    if K > len(out):
        raise ValueError("too many inputs for the drift table")
    return np.array(out[:K], dtype=np.int64)


def _extents(rng: Stream, npairs: int, axis_probs) -> np.ndarray:
    ext = np.zeros((npairs, 4), dtype=np.uint8)
    for a, pr in enumerate(axis_probs):
        if pr is None:
            continue
        ext[:, a] = rng.choice_p(pr, npairs).astype(np.uint8)
    return ext


def build_boxes(dims, drift: np.ndarray, ext_raw: np.ndarray, placement: str = "literal"):
    """Clamped successor boxes, per axis a with drift d and extent e:

    placement "literal": [x+d, x+d+e] on every axis;
    placement "drift":   [x+d, x+d+e] if d >= 0 and [x+d-e, x+d] if d < 0,
                         i.e. the spread extends in the direction of motion,
                         so a box never contains its own cell on the drift axis.
    Both corners are clamped into the grid (overflow cells of the cover are
    folded onto the border cells), so every F(x,u) is non-empty."""
    coords = cell_coords(dims)                     # [n,4]
    n = coords.shape[0]
    K = drift.shape[0]
    st = strides(dims)
    dimv = np.array(dims, dtype=np.int64)
    lo_lin = np.zeros(n * K, dtype=np.int64)
    ext = np.zeros((n * K, 4), dtype=np.uint8)
    for u in range(K):
        sel = slice(u, n * K, K)
        e = ext_raw[sel].astype(np.int64)
        d = drift[u][None, :]
        shift = np.where(d < 0, d - e, d) if placement == "drift" else np.broadcast_to(d, e.shape)
        lo_c = np.clip(coords + shift, 0, dimv[None, :] - 1)
        hi_c = np.clip(coords + shift + e, 0, dimv[None, :] - 1)
        lo_lin[sel] = (lo_c * st[None, :]).sum(axis=1)
        ext[sel] = (hi_c - lo_c).astype(np.uint8)
    return lo_lin.astype(np.uint32), ext


def _spatial_block_avoid(dims, rng: Stream, target: np.ndarray, frac: float, wmin=2, wmax=6,
                         span_axes=(2, 3)) -> np.ndarray:
    """Axis-aligned obstacle blocks over the spatial axes (0,1) that span the
    remaining axes entirely; added until >= frac of all cells, never
    intersecting the target footprint."""
    N0, N1 = dims[0], dims[1]
    tfoot = target.reshape(tuple(reversed(dims))).any(axis=(0, 1)) if len(dims) == 4 else None
    foot = np.zeros((N1, N0), dtype=bool)           # [x1, x0]
    goal = frac * N0 * N1
    tries = 0
    while foot.sum() < goal and tries < 100000:
        tries += 1
        w = int(rng.integers(wmin, wmax, 1)[0])
        h = int(rng.integers(wmin, wmax, 1)[0])
        a0 = int(rng.integers(0, max(0, N0 - w), 1)[0])
        a1 = int(rng.integers(0, max(0, N1 - h), 1)[0])
        blk = np.zeros_like(foot)
        blk[a1:a1 + h, a0:a0 + w] = True
        if (blk & tfoot).any():
            continue
        foot |= blk
    full = np.broadcast_to(foot[None, None, :, :], tuple(reversed(dims)))
    return full.reshape(-1).astype(np.uint8)


def grid_problem(dims, K: int, ext_probs, *, seed: int, dtype: str = "i32",
                 phi_top: float = 400.0, sigmas=(3.0, 3.0, 1.5, 1.5),
                 c_range=(1, 8), target_extent=None, avoid: str = "blocks",
                 avoid_frac: float = 0.05, with_csr: bool = True, name: str = "",
                 tilt=None, tilt_mix: float = 0.9, placement: str = "literal") -> Problem:
    """Generic grid instance (see module docstring).

    `tilt` (per-axis weights) adds a linear ramp to the potential before the
    rescale: phi = rescale((1-tilt_mix) * smooth + tilt_mix * ramp).  A ramp
    rising along every axis makes the boxes of the "+" drifts lie uphill of
    their cell, which is what produces many negative running costs."""
    dims = tuple(int(d) for d in dims) + (1,) * (4 - len(dims))
    ndim = sum(1 for d in dims if d > 1)
    n = int(np.prod(dims))
    drift = drifts_for(ndim, K)
    r_ext = Stream(seed, 1)
    r_tgt = Stream(seed, 2)
    r_av = Stream(seed, 3)
    r_phi = Stream(seed, 4)
    r_c = Stream(seed, 5)
    ext_raw = _extents(r_ext, n * K, ext_probs)
    lo, ext = build_boxes(dims, drift, ext_raw, placement)

    # target: a block of `target_extent` cells (full range on axes with extent None)
    coords = cell_coords(dims)
    te = list(target_extent) + [None] * (4 - len(target_extent))
    tmask = np.ones(n, dtype=bool)
    for a in range(4):
        if te[a] is None or dims[a] == 1:
            continue
        c0 = int(r_tgt.integers(0, dims[a] - te[a], 1)[0])
        tmask &= (coords[:, a] >= c0) & (coords[:, a] < c0 + te[a])

    if avoid == "iid":
        av = (r_av.uniform(n) < avoid_frac) & ~tmask
        av = av.astype(np.uint8)
    elif avoid == "blocks":
        av = _spatial_block_avoid(dims, r_av, tmask, avoid_frac)
    else:
        av = np.zeros(n, dtype=np.uint8)
    av[tmask] = 0

    if tilt is None:
        phi = smooth_field(dims, sigmas, r_phi, phi_top, integer=(dtype == "i32"))
    else:
        sm = smooth_field(dims, sigmas, r_phi, 1.0, integer=False)
        ramp = (coords.astype(np.float64) * np.asarray(tilt, dtype=np.float64)[None, :]).sum(axis=1)
        ramp /= max(ramp.max(), 1e-300)
        f = (1.0 - tilt_mix) * sm + tilt_mix * ramp
        f = (f - f.min()) / (f.max() - f.min()) * phi_top
        phi = np.rint(f).astype(np.int64) if dtype == "i32" else f
    mphi = box_min(dims, lo, ext, phi)
    phix = np.repeat(phi.astype(np.float64), K)
    if dtype == "i32":
        c = r_c.integers(c_range[0], c_range[1], n * K)
        gval = c + phix.astype(np.int64) - mphi.astype(np.int64)
        g = gval.astype(np.int32)
        G = np.where(tmask, 0, INF_I32).astype(np.int32)
        c_min = float(c_range[0])
    else:
        c = c_range[0] + (c_range[1] - c_range[0]) * r_c.uniform(n * K)
        g = (c + phix - mphi).astype(np.float32)
        G = np.where(tmask, np.float32(0.0), np.float32(np.inf)).astype(np.float32)
        c_min = float(c_range[0])
    prob = Problem(dims=dims, ndim=ndim, K=K, dtype=dtype, G=G, g=g, avoid=av,
                   box_lo=lo, box_ext=ext, target=tmask, phi=phi, cost_c=c, c_min=c_min,
                   name=name)
    if with_csr:
        prob.ensure_csr()
    return prob


# --------------------------------------------------------------------------
# The named workloads
# --------------------------------------------------------------------------
P_SPATIAL = (0.1, 0.3, 0.6)      # extent 0,1,2 on spatial axes
P_ANGULAR = (0.3, 0.7)           # extent 0,1 on heading / speed
P_HALF = (0.5, 0.5)              # extent 0,1 uniform


def grid2d_small(seed: Optional[int] = None, **kw) -> Problem:
    """2-D 64x64 grid, 4 inputs, extents {0,1}^2, 10% iid avoid, 4x4 target,
    int32 potential costs with phi in [0,40]."""
    s = instance_seed(1, 0) if seed is None else seed
    kw.setdefault("phi_top", 40.0)
    kw.setdefault("dtype", "i32")
    return grid_problem((64, 64), 4, [P_HALF, P_HALF], seed=s, sigmas=(3.0, 3.0, 0, 0),
                        target_extent=(4, 4), avoid="iid", avoid_frac=0.10,
                        name=f"grid2d_64x64_k4_{kw['dtype']}", **kw)


def grid4d(seed: Optional[int] = None, dtype: str = "i32", dims=(40, 40, 24, 10), K: int = 12,
           name: Optional[str] = None, **kw) -> Problem:
    """4-D UAV-style grid (x, y, heading, speed): 12 inputs, spatial extents
    {0,1,2}, angular {0,1}; 5% block obstacles; 3x3 spatial target slab.
    int32: c in U{1..8}, phi in [0,400].  fp32: c in U[0.5,4), phi in [0,300]."""
    s = instance_seed(2, 0) if seed is None else seed
    if dtype == "i32":
        kw.setdefault("phi_top", 400.0)
        kw.setdefault("c_range", (1, 8))
    else:
        kw.setdefault("phi_top", 300.0)
        kw.setdefault("c_range", (0.5, 4.0))
        kw.setdefault("tilt", (2.2, 2.2, 4.0, 4.0))
    nm = name or f"grid4d_{'x'.join(map(str, dims))}_k{K}_{dtype}"
    return grid_problem(dims, K, [P_SPATIAL, P_SPATIAL, P_ANGULAR, P_ANGULAR], seed=s, dtype=dtype,
                        sigmas=(3.0, 3.0, 1.5, 1.5), target_extent=(3, 3, None, None),
                        avoid="blocks", avoid_frac=0.05, name=nm, placement="drift", **kw)


def grid3d(seed: int, dims=(48, 48, 24), K: int = 6, **kw) -> Problem:
    kw.setdefault("phi_top", 200.0)
    return grid_problem(dims, K, [P_SPATIAL, P_SPATIAL, P_HALF], seed=seed, dtype="i32",
                        sigmas=(3.0, 3.0, 1.5, 0), target_extent=(3, 3, None),
                        avoid="blocks", avoid_frac=0.05, name=f"grid3d_{'x'.join(map(str, dims))}_k{K}",
                        placement="drift", **kw)


def grid2d(seed: int, dims=(128, 128), K: int = 4, **kw) -> Problem:
    kw.setdefault("phi_top", 40.0)
    return grid_problem(dims, K, [P_HALF, P_HALF], seed=seed, dtype="i32",
                        sigmas=(3.0, 3.0, 0, 0), target_extent=(4, 4), avoid="iid",
                        avoid_frac=0.10, name=f"grid2d_{'x'.join(map(str, dims))}_k{K}", **kw)


def batch_instance(i: int, count: int = 64, with_csr: bool = True) -> Problem:
    """Instance i of the uneven batch of `count` (see batch_mix)."""
    q = count // 4
    s = instance_seed(4, i)
    if i < q:
        return grid2d(s, with_csr=with_csr)
    if i < 2 * q:
        return grid3d(s, with_csr=with_csr)
    j = i - 2 * q
    nj = max(1, count - 2 * q - 1)
    t = j / nj
    dims = tuple(int(round(a + (b - a) * t)) for a, b in zip((20, 20, 12, 6), (40, 40, 24, 10)))
    K = 8 if (j % 2 == 0) else 12
    return grid4d(s, "i32", dims=dims, K=K, with_csr=with_csr)


def batch_mix(count: int = 64, with_csr: bool = True):
    """The uneven batch: 1/4 2-D 128x128 (K=4), 1/4 3-D 48x48x24 (K=6), 1/2
    4-D grids interpolated from 20x20x12x6 to 40x40x24x10 (K alternating 8/12)."""
    return [batch_instance(i, count, with_csr) for i in range(count)]


def learned_instance(index: int, with_csr: bool = True, dims=(60, 60, 30, 12)) -> Problem:
    """Learned-ordering workload: 60x60x30x12, 16 inputs, int32 costs.
    Training instances use indices 0..255, held-out ones 1000..1031."""
    return grid4d(instance_seed(5, index), "i32", dims=dims, K=16, with_csr=with_csr,
                  name=f"grid4d_{'x'.join(map(str, dims))}_k16_i32_#{index}")


# --------------------------------------------------------------------------
# Small explicit problems (not grids)
# --------------------------------------------------------------------------
def explicit_problem(n: int, K: int, rows, g, G, avoid=None, dtype="i32", name="") -> Problem:
    """Problem from explicit successor lists rows[x*K+u] (each non-empty)."""
    ptr = np.zeros(n * K + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([y for r in rows for y in sorted(r)], dtype=np.int32)
    if dtype == "i32":
        gg = np.array(g, dtype=np.int64)
        gg = np.where(gg >= INF_I32, INF_I32, gg).astype(np.int32)
        GG = np.array(G, dtype=np.int64)
        GG = np.where(GG >= INF_I32, INF_I32, GG).astype(np.int32)
    else:
        gg = np.array(g, dtype=np.float32)
        GG = np.array(G, dtype=np.float32)
    av = np.zeros(n, dtype=np.uint8) if avoid is None else np.asarray(avoid, dtype=np.uint8)
    return Problem(dims=(n, 1, 1, 1), ndim=1, K=K, dtype=dtype, G=GG, g=gg, avoid=av,
                   succ_ptr=ptr, succ_idx=idx, name=name)


def random_small(seed: int, n: int, K: int, max_succ: int = 3, cost_lo: int = -5, cost_hi: int = 5,
                 p_target: float = 0.4, p_forbid: float = 0.1, dtype: str = "i32") -> Problem:
    """Tiny random problem for brute-force comparisons: arbitrary successor
    sets of size 1..max_succ, integer costs in [cost_lo, cost_hi] (some
    inputs forbidden), random finite terminal costs on a random subset.
    May contain negative cycles; callers filter as they need."""
    r = Stream(seed, 11)
    rows = []
    for _ in range(n * K):
        k = int(r.integers(1, min(max_succ, n), 1)[0])
        perm = np.argsort(r.uniform(n))
        rows.append(sorted(int(v) for v in perm[:k]))
    g = r.integers(cost_lo, cost_hi, n * K)
    forbid = r.uniform(n * K) < p_forbid
    G = r.integers(cost_lo, cost_hi + 5, n)
    tgt = r.uniform(n) < p_target
    tgt[int(r.integers(0, n - 1, 1)[0])] = True
    if dtype == "i32":
        g = np.where(forbid, INF_I32, g)
        G = np.where(tgt, G, INF_I32)
    else:
        g = np.where(forbid, np.inf, g.astype(np.float64) + 0.25 * r.uniform(n * K))
        G = np.where(tgt, G.astype(np.float64), np.inf)
    return explicit_problem(n, K, rows, g, G, dtype=dtype, name=f"random_small_{seed}")


def potential_small(seed: int, n: int, K: int, max_succ: int = 3, dtype: str = "i32",
                    p_target: float = 0.3, zero_phi: bool = False) -> Problem:
    """Tiny random problem in potential form (no negative cycles)."""
    r = Stream(seed, 12)
    rows = []
    for _ in range(n * K):
        k = int(r.integers(1, min(max_succ, n), 1)[0])
        perm = np.argsort(r.uniform(n))
        rows.append(sorted(int(v) for v in perm[:k]))
    if dtype == "i32":
        phi = np.zeros(n, dtype=np.int64) if zero_phi else r.integers(0, 20, n)
        c = r.integers(1, 6, n * K)
        g = np.array([c[p] + phi[p // K] - min(phi[y] for y in rows[p]) for p in range(n * K)])
        G = np.where(r.uniform(n) < p_target, r.integers(0, 10, n), INF_I32)
    else:
        phi = np.zeros(n) if zero_phi else 20.0 * r.uniform(n)
        c = 0.5 + 3.0 * r.uniform(n * K)
        g = np.array([c[p] + phi[p // K] - min(phi[y] for y in rows[p]) for p in range(n * K)])
        G = np.where(r.uniform(n) < p_target, 10.0 * r.uniform(n), np.inf)
    if not np.any(np.asarray(G) < (INF_I32 if dtype == "i32" else np.inf)):
        G = np.array(G)
        G[0] = 0
    return explicit_problem(n, K, rows, g, G, dtype=dtype, name=f"potential_small_{seed}")


def with_edge_costs(prob: Problem, seed: int, extra=(0, 4), keep_pair=True) -> Problem:
    """The same system with per-edge running costs in potential form:
    h(x,y,u) = c'(x,y,u) + phi(x) - phi(y), c' drawn from `extra` (int32:
    U{lo..hi-1}; fp32: U[lo,hi)), and the per-pair part g(x,u) = c(x,u) (the
    positive part of the original cost; 0 if keep_pair is False).  Along any
    path the potential terms telescope, so every cycle costs at least its
    length times min c + min c' and no negative cycle exists (with c' >= 0
    and c >= c_min, or c' >= 1 when keep_pair is False).  Needs CSR rows
    and the potential phi."""
    import copy
    prob.ensure_csr()
    q = copy.copy(prob)
    r = Stream(seed, 21)
    ptr = np.asarray(prob.succ_ptr, dtype=np.int64)
    idx = np.asarray(prob.succ_idx, dtype=np.int64)
    m = int(ptr[-1])
    src = np.repeat(np.arange(prob.npairs, dtype=np.int64) // prob.K, np.diff(ptr))
    phi = np.asarray(prob.phi, dtype=np.float64)
    if prob.dtype == "i32":
        ce = r.integers(extra[0], extra[1], m)
        h = ce + phi[src].astype(np.int64) - phi[idx].astype(np.int64)
        q.g_edge = h.astype(np.int32)
        base = np.asarray(prob.cost_c, dtype=np.int64) if keep_pair else np.zeros(prob.npairs, np.int64)
        q.g = np.where(np.asarray(prob.g) >= INF_I32, INF_I32, base).astype(np.int32)
    else:
        ce = extra[0] + (extra[1] - extra[0]) * r.uniform(m)
        q.g_edge = (ce + phi[src] - phi[idx]).astype(np.float32)
        base = np.asarray(prob.cost_c, dtype=np.float64) if keep_pair else np.zeros(prob.npairs)
        q.g = np.where(np.isinf(np.asarray(prob.g)), np.inf, base).astype(np.float32)
    q.name = prob.name + "_edgecost"
    return q


def fire_region(prob: Problem, seed: int, size: int = 6) -> np.ndarray:
    """[n] bool: a planar block of cells (axes 0 and 1; size x size, at most
    a third of each axis) over all headings and the upper half of the
    speeds, away from the target: the stand-in for the paper's hot spot with
    its water-drop speed range (Sect. VI-A)."""
    N = prob.dims
    size = max(2, min(size, N[0] // 3, N[1] // 3))
    r = Stream(seed, 31)
    tgt = np.asarray(prob.G) == 0 if prob.dtype == "i32" else np.asarray(prob.G) == 0.0
    x = np.arange(prob.n, dtype=np.int64)
    c0, c1 = x % N[0], (x // N[0]) % N[1]
    c3 = x // (N[0] * N[1] * N[2])
    for _ in range(1000):
        f0 = int(r.integers(0, max(1, N[0] - size), 1)[0])
        f1 = int(r.integers(0, max(1, N[1] - size), 1)[0])
        reg = (c0 >= f0) & (c0 < f0 + size) & (c1 >= f1) & (c1 < f1 + size) & (c3 >= N[3] // 2)
        if not (reg & tgt).any():
            return reg & (np.asarray(prob.avoid) == 0)
    raise ValueError("no fire region away from the target")


def reward_problem(prob: Problem, V1: np.ndarray, seed: int, reward: int = 24) -> Problem:
    """The second problem of a chained mission (Sect. VI-A: fly to the hot
    spot, terminal cost G2 = V1 of the return problem), int32: the same
    system and per-pair costs g, terminal cost G2 = V1, and per-edge costs
    that reward entering the fire region and take the reward back on
    leaving it, h(x,y,u) = R (1[x in fire] - 1[y in fire]).  The per-edge
    part is a potential difference, so it telescopes along any path and adds
    no negative cycle to the potential-form g; the paper's own reward (a
    constant negative cost on every step into the region) would allow
    negative cycles on a synthetic grid.  The fire mask is kept as
    `fire`."""
    import copy
    assert prob.dtype == "i32"
    prob.ensure_csr()
    q = copy.copy(prob)
    fire = fire_region(prob, seed)
    ptr = np.asarray(prob.succ_ptr, dtype=np.int64)
    idx = np.asarray(prob.succ_idx, dtype=np.int64)
    src = np.repeat(np.arange(prob.npairs, dtype=np.int64) // prob.K, np.diff(ptr))
    f = fire.astype(np.int64)
    q.g_edge = (reward * (f[src] - f[idx])).astype(np.int32)
    q.g = np.asarray(prob.g, dtype=np.int32).copy()
    q.G = np.asarray(V1, dtype=np.int32).copy()
    q.fire = fire
    q.reward = reward
    q.name = prob.name + "_reward"
    return q


def potential_small_edges(seed: int, n: int, K: int, max_succ: int = 3, dtype: str = "i32",
                          p_target: float = 0.3, zero_phi: bool = False) -> Problem:
    """Tiny random problem with per-edge costs in potential form (no
    negative cycles; all costs >= 0 with zero_phi)."""
    prob = potential_small(seed, n, K, max_succ, dtype, p_target, zero_phi)
    r = Stream(seed, 22)
    phi = np.zeros(n) if zero_phi else (r.integers(0, 20, n) if dtype == "i32" else 20.0 * r.uniform(n))
    c = r.integers(1, 6, n * K) if dtype == "i32" else 0.5 + 3.0 * r.uniform(n * K)
    prob.phi = phi
    prob.cost_c = c
    return with_edge_costs(prob, seed, extra=(0, 4) if dtype == "i32" else (0.0, 2.0))


def random_small_edges(seed: int, n: int, K: int, max_succ: int = 3, lo: int = -5, hi: int = 5,
                       dtype: str = "i32") -> Problem:
    """random_small with arbitrary-sign per-edge costs h in [lo, hi) added
    to the per-pair costs.  May contain negative cycles."""
    prob = random_small(seed, n, K, max_succ, dtype=dtype)
    r = Stream(seed, 23)
    m = int(prob.succ_ptr[-1])
    if dtype == "i32":
        prob.g_edge = r.integers(lo, hi, m).astype(np.int32)
    else:
        prob.g_edge = (lo + (hi - lo) * r.uniform(m)).astype(np.float32)
    prob.name += "_edgecost"
    return prob


def chain_graph(seed: int, n: int, K: int, dtype: str = "i32") -> Problem:
    """Ordinary digraph as a system: every F(x,u) is a single state (|F|=1),
    the inputs select one of K out-edges.  Potential-form weights so that no
    negative cycle exists; a few terminal states."""
    r = Stream(seed, 13)
    succ = r.integers(0, n - 1, n * K)
    phi = r.integers(0, 30, n)
    c = r.integers(1, 9, n * K)
    g = c + np.repeat(phi, K) - phi[succ]
    G = np.where(r.uniform(n) < 0.05, r.integers(0, 20, n), INF_I32)
    G[int(r.integers(0, n - 1, 1)[0])] = 0
    rows = [[int(s)] for s in succ]
    return explicit_problem(n, K, rows, g, G, dtype=dtype, name=f"chain_{seed}")
