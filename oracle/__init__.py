"""CPU oracle for the generalized Bellman-Ford method — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the HIP library
(paper_2001_06231_amd); both are fed by the input generators in `synth`.

Contents
  gbf_oracle.c   Algorithm 1 of the paper (Sect. IV-A), single-threaded C,
                 plus the canonical policy / residual pass, a box decoder and
                 an independent min-max Dijkstra for non-negative costs;
                 running costs per pair, plus optional per-edge costs.
  brute.py       Brute force from the definitions of Sect. III: the operator
                 P, Kleene iteration, policy evaluation and enumeration of
                 memoryless strategies (tiny problems only).
  mlp_ref.py     fp64 reference of the frontier-ordering MLP.

Parity status: every function here is pinned by a `-m "not gpu"` test
(worked example of the paper, brute force, Dijkstra, classical
Bellman-Ford, invariants); see tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gbf_oracle.c")
_SRC_AC = os.path.join(_HERE, "aircraft.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, NEGCYCLE = 0, 1
HANDOVER, NONE = -1, -2
INF_I32 = 2**31 - 1

_lock = threading.Lock()
_lib = None


class Counters(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("pair_evals", ctypes.c_int64),
                ("edge_relax", ctypes.c_int64), ("improvements", ctypes.c_int64),
                ("saturations", ctypes.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def build() -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-o", tmp, _SRC, _SRC_AC, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _bind(L):
    """Declares the argument types of the oracle's entry points on L."""
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    for nm in ("oracle_solve_i32", "oracle_solve_f64", "oracle_solve_f32"):
        f = getattr(L, nm)
        f.argtypes = [i64, i64, P, P, P, P, P, P, i64, P, P, ctypes.POINTER(Counters), P, P]
        f.restype = ctypes.c_int
    for nm in ("oracle_policy_i32", "oracle_policy_f64", "oracle_policy_f32"):
        f = getattr(L, nm)
        f.argtypes = [i64, i64, P, P, P, P, P, P, P, P]
        f.restype = i64
    L.oracle_box_to_csr.argtypes = [P, i64, P, P, P]
    L.oracle_box_to_csr.restype = i64
    L.oracle_dijkstra_i32.argtypes = [i64, i64, P, P, P, P, P, P, P]
    L.oracle_dijkstra_i32.restype = ctypes.c_int
    L.oracle_residual_box_sample.argtypes = [P, i64, P, i64, P, P, P, P, P, P]
    L.oracle_residual_box_sample.restype = i64
    d = ctypes.c_double
    i32 = ctypes.c_int32
    for nm in ("oracle_ac_sin", "oracle_ac_cos"):
        getattr(L, nm).argtypes = [d]
        getattr(L, nm).restype = d
    L.oracle_ac_bank_rad.argtypes = [ctypes.c_int, ctypes.c_int, d]
    L.oracle_ac_bank_rad.restype = d
    L.oracle_ac_thrust.argtypes = [ctypes.c_int, ctypes.c_int, d]
    L.oracle_ac_thrust.restype = d
    L.oracle_ac_enclose.argtypes = [P, P, d, d, d, d, d, d, ctypes.c_int, P, P]
    L.oracle_ac_enclose.restype = ctypes.c_int
    L.oracle_ac_table.argtypes = [P, d, d, d, d, d, d, d, d, i32, i32, i32, d, d, P]
    L.oracle_ac_table.restype = i64
    return L


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
                    os.path.getmtime(_SRC), os.path.getmtime(_SRC_AC)):
                build()
            _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def build_variant(src_text: str, path: str, which: str = "solver") -> str:
    """Compiles a modified copy of one of the oracle's sources ("solver":
    gbf_oracle.c, "aircraft": aircraft.c) with the other unchanged; tests
    that plant a mistake in the oracle use this to show that a pin catches
    it."""
    src = path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    pair = [src, _SRC_AC] if which == "solver" else [_SRC, src]
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-o", path] + pair + ["-lm"])
    return path


class use_variant:
    """Context manager: the oracle's functions run on the library at `path`
    (built by build_variant) inside the block."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        lib()
        self._saved = _lib
        _lib = _bind(ctypes.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def source(which: str = "solver") -> str:
    with open(_SRC if which == "solver" else _SRC_AC) as f:
        return f.read()


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _inputs(prob):
    if prob.succ_ptr is None:
        ptr, idx = box_to_csr(prob.dims, prob.box_packed())
    else:
        ptr = np.ascontiguousarray(prob.succ_ptr, dtype=np.int64)
        idx = np.ascontiguousarray(prob.succ_idx, dtype=np.int32)
    av = np.ascontiguousarray(prob.avoid, dtype=np.uint8)
    return ptr, idx, av


def _edge_costs(prob, dtype):
    """Per-edge costs h (one per successor-list entry), or None."""
    h = getattr(prob, "g_edge", None)
    if h is None:
        return None
    if prob.succ_ptr is None:
        raise ValueError("per-edge costs need explicit successor lists")
    return np.ascontiguousarray(h, dtype=dtype)


def _precision(prob, precision):
    if prob.dtype == "i32":
        return "i32"
    return precision or "f64"


def solve(prob, precision: str | None = None, max_rounds: int = 0) -> dict:
    """Run Algorithm 1.  precision: 'i32' (int costs), 'f64' (default for
    float costs: the definition in double precision) or 'f32' (one single
    precision addition per backup).  Returns V, the Algorithm-1 mu, the
    canonical policy, the residual count, the status and the counters."""
    L = lib()
    prec = _precision(prob, precision)
    ptr, idx, av = _inputs(prob)
    n, K = prob.n, prob.K
    if prec == "i32":
        g = np.ascontiguousarray(prob.g, dtype=np.int32)
        G = np.ascontiguousarray(prob.G, dtype=np.int32)
        h = _edge_costs(prob, np.int32)
        W = np.empty(n, dtype=np.int32)
        fs, fp = L.oracle_solve_i32, L.oracle_policy_i32
    else:
        g = np.ascontiguousarray(prob.g, dtype=np.float32)
        G = np.ascontiguousarray(prob.G, dtype=np.float32)
        h = _edge_costs(prob, np.float32)
        W = np.empty(n, dtype=np.float64 if prec == "f64" else np.float32)
        fs, fp = (L.oracle_solve_f64, L.oracle_policy_f64) if prec == "f64" else \
                 (L.oracle_solve_f32, L.oracle_policy_f32)
    mu = np.empty(n, dtype=np.int32)
    c = Counters()
    front = np.empty(n, dtype=np.int32)
    flen = np.zeros(1, dtype=np.int64)
    st = fs(n, K, _p(ptr), _p(idx), _p(g), _p(h), _p(G), _p(av), int(max_rounds), _p(W), _p(mu),
            ctypes.byref(c), _p(front), _p(flen))
    if st < 0:
        raise ValueError(f"oracle rejected the problem (status {st})")
    pol = np.empty(n, dtype=np.int32)
    bad = fp(n, K, _p(ptr), _p(idx), _p(g), _p(h), _p(G), _p(av), _p(W), _p(pol))
    return {"V": W, "mu": mu, "policy": pol, "residual": int(bad), "status": int(st),
            "counters": c.as_dict(), "precision": prec, "frontier": front[:int(flen[0])].copy()}


def residual(prob, V, precision: str | None = None):
    """One application of P to V: returns (number of non-avoid states with
    P(V)(x) != V(x) or avoid states with finite V, canonical policy)."""
    L = lib()
    prec = _precision(prob, precision)
    ptr, idx, av = _inputs(prob)
    if prec == "i32":
        g = np.ascontiguousarray(prob.g, dtype=np.int32)
        G = np.ascontiguousarray(prob.G, dtype=np.int32)
        h = _edge_costs(prob, np.int32)
        W = np.ascontiguousarray(V, dtype=np.int32)
        f = L.oracle_policy_i32
    else:
        g = np.ascontiguousarray(prob.g, dtype=np.float32)
        G = np.ascontiguousarray(prob.G, dtype=np.float32)
        h = _edge_costs(prob, np.float32)
        W = np.ascontiguousarray(V, dtype=np.float64 if prec == "f64" else np.float32)
        f = L.oracle_policy_f64 if prec == "f64" else L.oracle_policy_f32
    pol = np.empty(prob.n, dtype=np.int32)
    bad = f(prob.n, prob.K, _p(ptr), _p(idx), _p(g), _p(h), _p(G), _p(av), _p(W), _p(pol))
    return int(bad), pol


def box_to_csr(dims, box: np.ndarray):
    """The oracle's own decoder of packed 8-byte boxes into CSR rows."""
    L = lib()
    d = np.ascontiguousarray(np.array(list(dims) + [1] * (4 - len(dims)), dtype=np.int32))
    b = np.ascontiguousarray(box, dtype=np.uint64)
    npairs = b.shape[0]
    m = L.oracle_box_to_csr(_p(d), npairs, _p(b), None, None)
    if m < 0:
        raise ValueError("box outside the grid")
    ptr = np.empty(npairs + 1, dtype=np.int64)
    idx = np.empty(m, dtype=np.int32)
    L.oracle_box_to_csr(_p(d), npairs, _p(b), _p(ptr), _p(idx))
    return ptr, idx


def residual_box_sample(dims, K, states, box_rows, g_rows, G_rows, avoid, V):
    """One application of P at the sampled states of an int32 box problem
    (gbf_oracle.c, oracle_residual_box_sample): `box_rows`/`g_rows` hold the
    K boxes and costs of each sampled state in order, `G_rows` its terminal
    cost, `avoid` and `V` are full arrays.  Returns (number of sampled states
    where P(V)(x) != V(x), the first offenders)."""
    L = lib()
    d = np.ascontiguousarray(np.array(list(dims) + [1] * (4 - len(dims)), dtype=np.int32))
    xs = np.ascontiguousarray(states, dtype=np.int64)
    b = np.ascontiguousarray(box_rows, dtype=np.uint64)
    g = np.ascontiguousarray(g_rows, dtype=np.int32)
    G = np.ascontiguousarray(G_rows, dtype=np.int32)
    av = np.ascontiguousarray(avoid, dtype=np.uint8)
    W = np.ascontiguousarray(V, dtype=np.int32)
    if b.size != xs.size * K or g.size != xs.size * K or G.size != xs.size:
        raise ValueError("one row of K boxes and costs, and one G, per sampled state")
    if xs.size and (xs.min() < 0 or xs.max() >= W.size):
        raise ValueError("sampled state out of range")
    out = np.zeros(16, dtype=np.int64)
    bad = L.oracle_residual_box_sample(_p(d), int(K), _p(xs), xs.size, _p(b), _p(g), _p(G), _p(av), _p(W), _p(out))
    if bad < 0:
        raise ValueError("box outside the grid")
    return int(bad), out[:min(int(bad), 16)].copy()


def dijkstra(prob) -> np.ndarray:
    """Independent min-max Dijkstra (int32, non-negative running costs)."""
    L = lib()
    ptr, idx, av = _inputs(prob)
    g = np.ascontiguousarray(prob.g, dtype=np.int32)
    G = np.ascontiguousarray(prob.G, dtype=np.int32)
    h = _edge_costs(prob, np.int32)
    W = np.empty(prob.n, dtype=np.int32)
    st = L.oracle_dijkstra_i32(prob.n, prob.K, _p(ptr), _p(idx), _p(g), _p(h), _p(G), _p(av), _p(W))
    if st != 0:
        raise ValueError(f"dijkstra rejected the problem (status {st})")
    return W
