"""gbf — generalized Bellman-Ford for symbolic optimal control on MI355X.

Thin ctypes binding of the C ABI in include/gbf.h (libgbf.so, built in-tree
by ``paper_2001_06231_amd.build``).  It only marshals arguments: every step
of the solve runs in the library's HIP kernels.  There is no CPU fallback;
if the library is missing, importing a function raises.

Names follow the paper (Weber, Kreuzer, Knoll, Sect. III-C and IV-A):
a problem is (X, U, F, G, g), the solver returns the value function V and a
controller (policy) that realizes it.

Use (arrays on the host or torch tensors on the GPU)::

    import paper_2001_06231_amd as gbf
    g = gbf.load_graph(n, K, G, g_pair, succ_ptr=ptr, succ_idx=idx, avoid=av)
    status, stats, V = g.solve()          # V: numpy, or pass V_out=<tensor>
    policy, residual = g.policy()         # -1 hand over, -2 no controller
    g.free()

``load_problem`` takes an object with those fields (see ``synth``) and an
encoding ("csr", "box", "box+rev", "box->csr", "box:budget");
``solve_batch`` solves many handles in one frontier; ``MLP`` is the
frontier-ordering network (keys for ``solve(order="buckets", ...)``).
"""
from __future__ import annotations

import atexit
import ctypes
import os
import threading
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgbf.so")

# status codes and constants of include/gbf.h
OK, ENEGCYCLE, EINVAL, ENOMEM, EHIP, ENOTSOLVED, ETIMEOUT = 0, 1, -1, -2, -3, -4, -5
I32, F32 = 0, 1
CSR, BOX = 0, 1
HOST, DEVICE = 0, 1
ORDER_PLAIN, ORDER_BUCKETS = 0, 1
MODE_AUTO, MODE_HOSTLOOP, MODE_PERSISTENT, MODE_SINGLE_BLOCK = 0, 1, 2, 3
HANDOVER, NONE = -1, -2
INF_I32 = 2**31 - 1
NOALLOC_MAX_PAIRS, NOALLOC_MAX_ROUNDS = 1 << 23, 1 << 21

_MODES = {"auto": MODE_AUTO, "hostloop": MODE_HOSTLOOP, "persistent": MODE_PERSISTENT,
          "single_block": MODE_SINGLE_BLOCK}
_ORDERS = {"plain": ORDER_PLAIN, "buckets": ORDER_BUCKETS}


class GbfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gbf error {code}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int64), ("n_inputs", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("encoding", ctypes.c_int32), ("memspace", ctypes.c_int32), ("G", ctypes.c_void_p),
                ("g", ctypes.c_void_p), ("avoid", ctypes.c_void_p), ("succ_ptr", ctypes.c_void_p),
                ("succ_idx", ctypes.c_void_p), ("dims", ctypes.c_int32 * 4), ("box", ctypes.c_void_p),
                ("expand_box", ctypes.c_int32), ("pair_ids64", ctypes.c_int32), ("g_edge", ctypes.c_void_p),
                ("mem_budget", ctypes.c_int64)]


class _Opts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("mode", ctypes.c_int32), ("bucket_key", ctypes.c_void_p),
                ("max_rounds", ctypes.c_int64), ("lanes", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("v_memspace", ctypes.c_int32), ("profile", ctypes.c_int32), ("batch_hint", ctypes.c_int32),
                ("bucket_span", ctypes.c_int32), ("bucket_budget", ctypes.c_int32), ("mem_floor_mib", ctypes.c_int32),
                ("block", ctypes.c_int32), ("compact_grid", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("fallback", ctypes.c_int32), ("rounds", ctypes.c_int64),
                ("pair_evals", ctypes.c_int64), ("edge_relax", ctypes.c_int64),
                ("improvements", ctypes.c_int64), ("saturations", ctypes.c_int64),
                ("expansions", ctypes.c_int64), ("marks", ctypes.c_int64),
                ("solve_ms", ctypes.c_double), ("relax_ms", ctypes.c_double),
                ("relax_launches", ctypes.c_int64), ("barrier_ms", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("mode_used", ctypes.c_int32), ("grid_used", ctypes.c_int32), ("block_used", ctypes.c_int32),
                ("lanes_used", ctypes.c_int32), ("graph_used", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("enc_used", ctypes.c_int32), ("images_dropped", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


EXPORTS = ("gbf_load_graph", "gbf_solve", "gbf_extract_policy", "gbf_solve_batch", "gbf_tune", "gbf_free_graph",
           "gbf_last_error", "gbf_shutdown", "gbf_solve_noalloc", "gbf_mlp_create", "gbf_mlp_set_params", "gbf_mlp_get_params", "gbf_mlp_samples",
           "gbf_mlp_forward", "gbf_mlp_grad", "gbf_mlp_train_step", "gbf_mlp_bucket_keys", "gbf_mlp_free",
           "gbf_aircraft_table", "gbf_load_aircraft")
MLP_NPARAMS = 4545

_lock = threading.Lock()
_lib = None
# live handles (graphs, networks): released by the exit handler below while
# the HIP runtime is still up; afterwards every release is a no-op
_live = weakref.WeakSet()
_closed = False


def _shutdown():
    """Exit handler: frees every live handle and the library's batch state
    (captured graphs, streams) before the HIP runtime shuts down."""
    global _closed
    if _closed or _lib is None:
        _closed = True
        return
    for obj in list(_live):
        try:
            obj.free()
        except Exception:
            pass
    _lib.gbf_shutdown()
    _closed = True


class _AcBox(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 4), ("hi", ctypes.c_int32 * 4)]


class _Aircraft(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("x_max", ctypes.c_int32 * 2), ("v_range", ctypes.c_int32 * 2),
                ("mass", ctypes.c_double), ("p_D", ctypes.c_double), ("p_L", ctypes.c_double),
                ("tau", ctypes.c_double), ("steps", ctypes.c_int32), ("n_thrust", ctypes.c_int32),
                ("n_bank", ctypes.c_int32), ("thrust_max", ctypes.c_double), ("bank_max_deg", ctypes.c_double),
                ("target", ctypes.POINTER(_AcBox)), ("n_target", ctypes.c_int32),
                ("avoid", ctypes.POINTER(_AcBox)), ("n_avoid", ctypes.c_int32),
                ("reward", ctypes.POINTER(_AcBox)), ("n_reward", ctypes.c_int32),
                ("reward_cost", ctypes.c_float), ("G", ctypes.c_void_p), ("pair_ids64", ctypes.c_int32)]


def lib():
    """Loads libgbf.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python paper_2001_06231_amd/build.py`")
            L = ctypes.CDLL(LIB_PATH)
            P = ctypes.c_void_p
            L.gbf_load_graph.argtypes = [ctypes.POINTER(_Problem), P, ctypes.POINTER(P)]
            L.gbf_load_graph.restype = ctypes.c_int
            L.gbf_solve.argtypes = [P, ctypes.POINTER(_Opts), P, ctypes.POINTER(_Stats)]
            L.gbf_solve.restype = ctypes.c_int
            L.gbf_solve_noalloc.argtypes = [P, ctypes.POINTER(_Opts), P, ctypes.POINTER(_Stats)]
            L.gbf_solve_noalloc.restype = ctypes.c_int
            L.gbf_extract_policy.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
            L.gbf_extract_policy.restype = ctypes.c_int
            L.gbf_solve_batch.argtypes = [ctypes.POINTER(P), ctypes.c_int32, ctypes.POINTER(_Opts),
                                          ctypes.POINTER(P), P]
            L.gbf_solve_batch.restype = ctypes.c_int
            L.gbf_tune.argtypes = [ctypes.POINTER(P), ctypes.c_int32, ctypes.POINTER(_Opts), ctypes.c_int32,
                                   ctypes.POINTER(_Opts), ctypes.POINTER(ctypes.c_double)]
            L.gbf_tune.restype = ctypes.c_int
            L.gbf_free_graph.argtypes = [P]
            L.gbf_free_graph.restype = None
            L.gbf_last_error.argtypes = []
            L.gbf_last_error.restype = ctypes.c_char_p
            L.gbf_shutdown.argtypes = []
            L.gbf_shutdown.restype = None
            I64, F, I = ctypes.c_int64, ctypes.c_float, ctypes.c_int32
            D4 = ctypes.POINTER(ctypes.c_int32)
            for name, args in (
                    ("gbf_mlp_create", [P, P, ctypes.POINTER(P)]),
                    ("gbf_mlp_set_params", [P, P]),
                    ("gbf_mlp_get_params", [P, P, P]),
                    ("gbf_mlp_samples", [P, D4, F, F, P, I, F, P, I64, P, P]),
                    ("gbf_mlp_forward", [P, P, I64, P]),
                    ("gbf_mlp_grad", [P, P, P, I64, P, I64, P, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(I64)]),
                    ("gbf_mlp_train_step", [P, P, P, I64, P, I64, F, ctypes.POINTER(F)]),
                    ("gbf_mlp_bucket_keys", [P, D4, F, F, F, F, P, P, ctypes.POINTER(F)])):
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
            L.gbf_mlp_free.argtypes = [P]
            L.gbf_mlp_free.restype = None
            L.gbf_aircraft_table.argtypes = [ctypes.POINTER(_Aircraft), P, P]
            L.gbf_aircraft_table.restype = ctypes.c_int
            L.gbf_load_aircraft.argtypes = [ctypes.POINTER(_Aircraft), P, ctypes.POINTER(P)]
            L.gbf_load_aircraft.restype = ctypes.c_int
            _lib = L
            # registered after torch's own handlers, so it runs before them
            atexit.register(_shutdown)
    return _lib


def _err(L, code):
    return GbfError(code, L.gbf_last_error().decode())


def _ptr(a):
    """Address and memory space of a numpy array or a torch tensor."""
    if a is None:
        return None, None
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return a.ctypes.data, HOST
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return a.data_ptr(), (DEVICE if a.is_cuda else HOST)
    raise TypeError(f"unsupported array type {type(a)}")


def current_stream():
    """The current torch HIP stream as a raw handle (None = default)."""
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class Graph:
    """A loaded problem (device-resident); see gbf_load_graph."""

    def __init__(self, handle, n, K, dtype, keep):
        self._h = handle
        self.n, self.K, self.dtype = n, K, dtype
        self._keep = keep
        _live.add(self)

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "_h", None):
            L = _lib
            if L is not None and not _closed:
                L.gbf_free_graph(self._h)
            self._h = None

    def _opts(self, order, mode, max_rounds, grid, profile, bucket_key, v_space, lanes=0, bucket_span=0,
              bucket_budget=0, mem_floor_mib=0, block=0, compact_grid=0):
        o = _Opts()
        o.mem_floor_mib = int(mem_floor_mib)
        o.block = int(block)
        o.compact_grid = int(compact_grid)
        o.lanes = int(lanes)
        o.bucket_span = int(bucket_span)
        o.bucket_budget = int(bucket_budget)
        o.order = _ORDERS[order]
        o.mode = _MODES[mode]
        o.max_rounds = int(max_rounds)
        o.grid = int(grid)
        o.profile = 1 if profile else 0
        o.v_memspace = v_space
        if bucket_key is not None:
            if bucket_key.element_size() != 2 or bucket_key.numel() < self.n:
                raise ValueError("bucket_key must hold n 16-bit keys")
            o.bucket_key, sp = _ptr(bucket_key)
            if sp != DEVICE:
                raise ValueError("bucket_key must be a device tensor")
        return o

    def solve(self, V_out=None, *, order="plain", mode="auto", max_rounds=0, grid=0, profile=False,
              bucket_key=None, lanes=0, bucket_span=0, bucket_budget=0, mem_floor_mib=0, block=0, compact_grid=0,
              check=True):
        """Runs the solver; returns (status, stats dict, V_out).  V_out may be
        a numpy array (host) or a torch tensor on the GPU; if None a numpy
        array is allocated."""
        L = lib()
        if V_out is None:
            V_out = np.empty(self.n, dtype=np.int32 if self.dtype == I32 else np.float32)
        vp, vs = _ptr(V_out)
        o = self._opts(order, mode, max_rounds, grid, profile, bucket_key, vs, lanes, bucket_span, bucket_budget,
                       mem_floor_mib, block, compact_grid)
        st = _Stats()
        rc = L.gbf_solve(self._h, ctypes.byref(o), vp, ctypes.byref(st))
        if rc < 0 or (check and rc not in (OK, ENEGCYCLE)):
            raise _err(L, rc)
        return rc, st.as_dict(), V_out

    def solve_noalloc(self, V_out=None, *, mode="auto", max_rounds=0, grid=0, lanes=0, block=0, compact_grid=0,
                      check=True):
        """gbf_solve_noalloc: the plain-order solve with all scratch in the
        library's static device array (no allocation in the call).  Returns
        (status, stats dict, V_out) as solve()."""
        L = lib()
        if V_out is None:
            V_out = np.empty(self.n, dtype=np.int32 if self.dtype == I32 else np.float32)
        vp, vs = _ptr(V_out)
        o = self._opts("plain", mode, max_rounds, grid, False, None, vs, lanes, 0, 0, 0, block, compact_grid)
        st = _Stats()
        rc = L.gbf_solve_noalloc(self._h, ctypes.byref(o), vp, ctypes.byref(st))
        if rc < 0 or (check and rc not in (OK, ENEGCYCLE)):
            raise _err(L, rc)
        return rc, st.as_dict(), V_out

    def policy(self, out=None):
        """Canonical controller of the last solve and the fixed-point
        residual count: (policy, residual)."""
        L = lib()
        if out is None:
            out = np.empty(self.n, dtype=np.int32)
        pp, ps = _ptr(out)
        res = ctypes.c_int64(0)
        rc = L.gbf_extract_policy(self._h, pp, ps, ctypes.byref(res))
        if rc != OK:
            raise _err(L, rc)
        return out, int(res.value)


def load_graph(n, K, G, g, *, dtype="i32", encoding="csr", avoid=None, succ_ptr=None, succ_idx=None,
               dims=None, box=None, expand_box=False, g_edge=None, mem_budget=0, pair_ids64=False,
               stream=None) -> Graph:
    """gbf_load_graph.  Arrays are numpy (host) or torch tensors on the GPU
    (all of one kind).  G/g (and the optional per-edge costs g_edge, CSR
    only) are int32 or float32 bit patterns."""
    L = lib()
    p = _Problem()
    p.n_states = int(n)
    p.n_inputs = int(K)
    p.dtype = I32 if dtype == "i32" else F32
    p.encoding = CSR if encoding == "csr" else BOX
    keep = []
    spaces = set()

    def put(field, arr, np_dtype):
        if arr is None:
            return
        if isinstance(arr, np.ndarray):
            arr = np.ascontiguousarray(arr, dtype=np_dtype)
        keep.append(arr)
        ptr, sp = _ptr(arr)
        spaces.add(sp)
        setattr(p, field, ptr)

    vt = np.int32 if dtype == "i32" else np.float32
    put("G", G, vt)
    put("g", g, vt)
    put("avoid", avoid, np.uint8)
    if p.encoding == CSR:
        put("succ_ptr", succ_ptr, np.int64)
        put("succ_idx", succ_idx, np.int32)
        put("g_edge", g_edge, vt)
    else:
        if g_edge is not None:
            raise ValueError("per-edge costs need the csr encoding")
        put("box", box, np.uint64)
        d = list(dims) + [1] * (4 - len(dims))
        for a in range(4):
            p.dims[a] = int(d[a])
        p.expand_box = int(expand_box)
        p.mem_budget = int(mem_budget)
    p.pair_ids64 = 1 if pair_ids64 else 0
    if len(spaces) > 1:
        raise ValueError("problem arrays must all be host arrays or all device tensors")
    p.memspace = spaces.pop() if spaces else HOST
    h = ctypes.c_void_p()
    rc = L.gbf_load_graph(ctypes.byref(p), stream, ctypes.byref(h))
    if rc != OK:
        raise _err(L, rc)
    return Graph(h, int(n), int(K), p.dtype, None)


def _aircraft(scn, G=None, pair_ids64=False):
    """A gbf_aircraft struct for a scenario with the fields of
    synth.aircraft.Scenario (and the arrays it points to)."""
    a = _Aircraft()
    for k in range(4):
        a.dims[k] = int(scn.dims[k])
    for k in range(2):
        a.x_max[k] = int(scn.x_max[k])
        a.v_range[k] = int(scn.v_range[k])
    a.mass, a.p_D, a.p_L, a.tau = float(scn.mass), float(scn.p_D), float(scn.p_L), float(scn.tau)
    a.steps, a.n_thrust, a.n_bank = int(scn.steps), int(scn.n_thrust), int(scn.n_bank)
    a.thrust_max, a.bank_max_deg = float(scn.thrust_max), float(scn.bank_max_deg)
    keep = []
    for name in ("target", "avoid", "reward"):
        boxes = list(getattr(scn, name))
        arr = (_AcBox * max(1, len(boxes)))()
        for i, (lo, hi) in enumerate(boxes):
            for k in range(4):
                arr[i].lo[k], arr[i].hi[k] = int(lo[k]), int(hi[k])
        keep.append(arr)
        setattr(a, name, ctypes.cast(arr, ctypes.POINTER(_AcBox)))
        setattr(a, "n_" + name, len(boxes))
    a.reward_cost = float(scn.reward_cost)
    a.pair_ids64 = 1 if pair_ids64 else 0
    if G is not None:
        ptr, sp = _ptr(G)
        if sp != DEVICE or G.dtype.itemsize != 4 or G.numel() != int(np.prod(scn.dims)):
            raise ValueError("G must be a float32 device tensor with one value per cell")
        keep.append(G)
        a.G = ptr
    return a, keep


def aircraft_table(scn, stream=None):
    """gbf_aircraft_table: the enclosure table as an int32 device tensor
    [dims[3], dims[2], K, 8]."""
    import torch
    L = lib()
    a, keep = _aircraft(scn)
    out = torch.empty((scn.dims[3], scn.dims[2], scn.n_thrust * scn.n_bank, 8), dtype=torch.int32, device="cuda")
    rc = L.gbf_aircraft_table(ctypes.byref(a), out.data_ptr(), stream)
    if rc != OK:
        raise _err(L, rc)
    return out


def load_aircraft(scn, G=None, stream=None, pair_ids64=False) -> Graph:
    """gbf_load_aircraft: the abstraction of a scenario, built on the device.
    G (float32 device tensor over the cells, e.g. the values of a first
    problem) replaces the target sets as terminal cost; pair_ids64 asks for
    64-bit pair ids at any size."""
    L = lib()
    a, keep = _aircraft(scn, G, pair_ids64)
    h = ctypes.c_void_p()
    rc = L.gbf_load_aircraft(ctypes.byref(a), stream, ctypes.byref(h))
    if rc != OK:
        raise _err(L, rc)
    return Graph(h, int(np.prod(scn.dims)), int(scn.n_thrust * scn.n_bank), F32, None)


def load_problem(prob, encoding="csr", stream=None, mem_budget=0, pair_ids64=False) -> Graph:
    """Loads an object with the fields of an optimal control problem
    (n, K, dtype, G, g, avoid, succ_ptr/succ_idx or dims/box_packed(), and
    optionally per-edge costs g_edge in succ_idx order).
    encoding: "csr" (explicit lists; expanded from the boxes on the device
    when the object carries no lists), "box" (implicit), "box->csr" or
    "box+rev" (box successors, reverse CSR for the predecessors), or
    "box:budget" ("box+rev" if the predecessor images fit `mem_budget`
    bytes, 0 = 68% of the free device memory, else "box").  Per-edge costs
    need "csr" with explicit lists."""
    g_edge = getattr(prob, "g_edge", None)
    if g_edge is not None:
        if encoding != "csr" or getattr(prob, "succ_ptr", None) is None:
            raise ValueError("per-edge costs need the csr encoding with explicit successor lists")
        return load_graph(prob.n, prob.K, prob.G, prob.g, dtype=prob.dtype, encoding="csr", avoid=prob.avoid,
                          succ_ptr=prob.succ_ptr, succ_idx=prob.succ_idx, g_edge=g_edge, stream=stream)
    if encoding == "box:budget":
        return load_graph(prob.n, prob.K, prob.G, prob.g, dtype=prob.dtype, encoding="box", avoid=prob.avoid,
                          dims=prob.dims, box=prob.box_packed(), expand_box=3, mem_budget=mem_budget,
                          pair_ids64=pair_ids64, stream=stream)
    if encoding == "box+rev":
        return load_graph(prob.n, prob.K, prob.G, prob.g, dtype=prob.dtype, encoding="box", avoid=prob.avoid,
                          dims=prob.dims, box=prob.box_packed(), expand_box=2, pair_ids64=pair_ids64,
                          stream=stream)
    if encoding == "box->csr" or (encoding == "csr" and getattr(prob, "succ_ptr", None) is None):
        return load_graph(prob.n, prob.K, prob.G, prob.g, dtype=prob.dtype, encoding="box", avoid=prob.avoid,
                          dims=prob.dims, box=prob.box_packed(), expand_box=1, pair_ids64=pair_ids64,
                          stream=stream)
    if encoding == "csr":
        return load_graph(prob.n, prob.K, prob.G, prob.g, dtype=prob.dtype, encoding="csr", avoid=prob.avoid,
                          succ_ptr=prob.succ_ptr, succ_idx=prob.succ_idx, stream=stream)
    return load_graph(prob.n, prob.K, prob.G, prob.g, dtype=prob.dtype, encoding="box", avoid=prob.avoid,
                      dims=prob.dims, box=prob.box_packed(), pair_ids64=pair_ids64, stream=stream)


def solve_batch(graphs: Sequence[Graph], V_outs=None, *, mode="auto", max_rounds=0, grid=0, profile=False,
                lanes=0, block=0, compact_grid=0, check=True):
    """gbf_solve_batch: one frontier over all instances.  Returns (worst
    status, list of per-instance stats, V_outs)."""
    L = lib()
    cnt = len(graphs)
    if V_outs is None:
        V_outs = [np.empty(gr.n, dtype=np.int32 if gr.dtype == I32 else np.float32) for gr in graphs]
    ptrs = [_ptr(v) for v in V_outs]
    spaces = {sp for _, sp in ptrs}
    if len(spaces) != 1:
        raise ValueError("V_outs must all be host or all device")
    o = _Opts()
    o.mode = _MODES[mode]
    o.max_rounds = int(max_rounds)
    o.grid = int(grid)
    o.lanes = int(lanes)
    o.block = int(block)
    o.compact_grid = int(compact_grid)
    o.profile = 1 if profile else 0
    o.v_memspace = spaces.pop()
    hs = (ctypes.c_void_p * cnt)(*[gr._h for gr in graphs])
    vs = (ctypes.c_void_p * cnt)(*[p for p, _ in ptrs])
    st = (_Stats * cnt)()
    rc = L.gbf_solve_batch(hs, cnt, ctypes.byref(o), vs, st)
    if rc < 0 or (check and rc not in (OK, ENEGCYCLE)):
        raise _err(L, rc)
    return rc, [s.as_dict() for s in st], V_outs


_MODE_NAMES = {v: k for k, v in _MODES.items()}  # includes "single_block"


def tune(graphs: Sequence[Graph], reps=3, order="plain", bucket_key=None, bucket_span=0, mode="auto"):
    """gbf_tune: the fastest launch configuration for these handles (one
    instance, or a batch), over every mode or within `mode`.  Returns
    (options dict for Graph.solve / solve_batch, median solve ms)."""
    L = lib()
    cnt = len(graphs)
    base = graphs[0]._opts(order, mode, 0, 0, False, bucket_key, DEVICE, 0, bucket_span)
    best = _Opts()
    ms = ctypes.c_double(0.0)
    hs = (ctypes.c_void_p * cnt)(*[gr._h for gr in graphs])
    rc = L.gbf_tune(hs, cnt, ctypes.byref(base), int(reps), ctypes.byref(best), ctypes.byref(ms))
    if rc != OK:
        raise _err(L, rc)
    return {"mode": _MODE_NAMES[best.mode], "lanes": best.lanes, "grid": best.grid, "block": best.block,
            "compact_grid": best.compact_grid}, ms.value


# ---------------------------------------------------------------------------
# Frontier-ordering network (gbf_mlp_*)
# ---------------------------------------------------------------------------
def _dev_ptr(t, what, dtype_size=None, numel=None):
    if t is None:
        return None
    if not hasattr(t, "is_cuda") or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous device tensor")
    if dtype_size is not None and t.element_size() != dtype_size:
        raise ValueError(f"{what} has the wrong element size")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{what} is too small")
    return t.data_ptr()


def _dims4(dims):
    d = list(dims) + [1] * (4 - len(dims))
    return (ctypes.c_int32 * 4)(*[int(v) for v in d])


class MLP:
    """The frontier-ordering network (gbf_mlp_*): 4 -> 64 -> 64 -> 1, bf16
    working weights, fp32 master weights trained with Adam.  Device arrays
    are torch tensors on the GPU; work runs on `stream` (default: torch's
    current stream)."""

    def __init__(self, params, stream=None):
        L = lib()
        self._stream = current_stream() if stream is None else stream
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_NPARAMS,):
            raise ValueError(f"params must have {MLP_NPARAMS} entries")
        h = ctypes.c_void_p()
        rc = L.gbf_mlp_create(p.ctypes.data, self._stream, ctypes.byref(h))
        if rc != OK:
            raise _err(L, rc)
        self._h = h
        _live.add(self)

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "_h", None):
            if _lib is not None and not _closed:
                _lib.gbf_mlp_free(self._h)
            self._h = None

    def _check(self, rc):
        if rc != OK:
            raise _err(lib(), rc)

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (MLP_NPARAMS,):
            raise ValueError(f"params must have {MLP_NPARAMS} entries")
        self._check(lib().gbf_mlp_set_params(self._h, p.ctypes.data))

    def params(self):
        """(fp32 master copy, bf16 working copy as uint16 bit patterns)."""
        m = np.empty(MLP_NPARAMS, np.float32)
        b = np.empty(MLP_NPARAMS, np.uint16)
        self._check(lib().gbf_mlp_get_params(self._h, m.ctypes.data, b.ctypes.data))
        return m, b

    def samples(self, dims, tc, cells, V=None, scale=1000.0):
        """Features (and labels V/scale if V is given) of the cells."""
        import torch
        cnt = int(cells.numel())
        feat = torch.empty((cnt, 4), dtype=torch.float32, device=cells.device)
        tgt = torch.empty(cnt, dtype=torch.float32, device=cells.device) if V is not None else None
        vdt = (F32 if V.dtype == torch.float32 else I32) if V is not None else I32
        self._check(lib().gbf_mlp_samples(self._h, _dims4(dims), float(tc[0]), float(tc[1]),
                                          _dev_ptr(V, "V", 4), vdt, float(scale),
                                          _dev_ptr(cells, "cells", 8), cnt, _dev_ptr(feat, "feat"),
                                          _dev_ptr(tgt, "target")))
        return feat, tgt

    def forward(self, feat):
        import torch
        cnt = int(feat.shape[0])
        out = torch.empty(cnt, dtype=torch.float32, device=feat.device)
        self._check(lib().gbf_mlp_forward(self._h, _dev_ptr(feat, "feat", 4, 4 * cnt), cnt, _dev_ptr(out, "out")))
        return out

    def grad(self, feat, target, idx=None):
        rows = int(target.numel())
        cnt = int(idx.numel()) if idx is not None else rows
        g = np.empty(MLP_NPARAMS, np.float32)
        loss = ctypes.c_double(0.0)
        lab = ctypes.c_int64(0)
        self._check(lib().gbf_mlp_grad(self._h, _dev_ptr(feat, "feat", 4, 4 * rows), _dev_ptr(target, "target", 4),
                                       rows, _dev_ptr(idx, "idx", 8), cnt, g.ctypes.data, ctypes.byref(loss),
                                       ctypes.byref(lab)))
        return g, loss.value, lab.value

    def train_step(self, feat, target, idx=None, lr=1e-3, want_loss=False):
        rows = int(target.numel())
        cnt = int(idx.numel()) if idx is not None else rows
        loss = ctypes.c_float(0.0)
        self._check(lib().gbf_mlp_train_step(self._h, _dev_ptr(feat, "feat", 4, 4 * rows),
                                             _dev_ptr(target, "target", 4), rows, _dev_ptr(idx, "idx", 8), cnt,
                                             float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def bucket_keys(self, dims, tc, scale=1000.0, width=16.0, keys=None, vhat=None):
        """Bucket keys of every cell (device int16 tensor holding the uint16
        keys, for Graph.solve(order="buckets", bucket_key=...)) and the
        minimum prediction."""
        import torch
        n = int(np.prod([int(v) for v in dims]))
        if keys is None:
            keys = torch.empty(n, dtype=torch.int16, device="cuda")
        vmin = ctypes.c_float(0.0)
        self._check(lib().gbf_mlp_bucket_keys(self._h, _dims4(dims), float(tc[0]), float(tc[1]), float(scale),
                                              float(width), _dev_ptr(keys, "keys", 2, n),
                                              _dev_ptr(vhat, "vhat", 4, n), ctypes.byref(vmin)))
        return keys, vmin.value
