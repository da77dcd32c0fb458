"""Brute force from the paper's definitions — TEST INFRASTRUCTURE ONLY.

These functions restate Sect. III of the paper directly and are used to pin
the C oracle (Algorithm 1) to something other than itself:

  apply_P       the dynamic programming operator of Sect. III-C,
                P(W)(x) = min{G(x), min_u max_{y in F(x,u)} g(x,y,u) + W(y)},
                with g(x,y,u) = g(x,u) + h(x,y,u) (h = 0 without per-edge
                costs), in exact Python arithmetic (ints, or floats with
                math.inf).
  kleene        its iterates P^k(G) from the top; V is the limit (the maximal
                fixed point, Theorem on dynamic programming, Sect. III-C).
  evaluate      closed-loop performance L(., mu) of a memoryless controller
                (Sect. III-B): the maximal fixed point of the operator of the
                system restricted to the controller's inputs; for a hand-over
                state the value is G(x).
  enumerate_V   V(p) = inf over controllers of L(p, mu) (definition of the
                value function, Sect. III-C), by enumerating every
                deterministic memoryless controller (tiny problems only).
  cost_J        the cost functional J(u, v, x) of Sect. III-B for explicit
                signals.
  kleene_np     the same Kleene iteration vectorised with numpy over CSR rows
                (moderate sizes); float64 or float32 arithmetic as requested.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

INF = math.inf
INF_I32 = 2**31 - 1


class Diverged(Exception):
    """The iteration did not reach a fixed point: some value tends to -inf."""


def _vals(prob):
    """(G, g, rows, avoid): rows[p] lists (y, h) for y in F(x,u), with h the
    per-edge part of the running cost g(x,y,u) = g(x,u) + h (0 if the
    problem has no per-edge costs)."""
    if prob.dtype == "i32":
        G = [INF if int(v) >= INF_I32 else int(v) for v in prob.G]
        g = [INF if int(v) >= INF_I32 else int(v) for v in prob.g]
    else:
        G = [float(v) for v in prob.G]
        g = [float(v) for v in prob.g]
    he = getattr(prob, "g_edge", None)
    if he is None:
        hv = [0] * int(prob.succ_ptr[-1])
    elif prob.dtype == "i32":
        hv = [int(v) for v in he]
    else:
        hv = [float(v) for v in he]
    rows = [[(int(prob.succ_idx[e]), hv[e]) for e in range(int(prob.succ_ptr[p]), int(prob.succ_ptr[p + 1]))]
            for p in range(prob.npairs)]
    avoid = [bool(a) for a in prob.avoid]
    return G, g, rows, avoid


def apply_P(prob, W, _cache=None):
    G, g, rows, avoid = _cache or _vals(prob)
    K = prob.K
    out = []
    for x in range(prob.n):
        if avoid[x]:
            out.append(INF)
            continue
        best = G[x]
        for u in range(K):
            p = x * K + u
            d = max(g[p] + h + W[y] for y, h in rows[p])
            if d < best:
                best = d
        out.append(best)
    return out


def kleene(prob, max_iter=None):
    """Iterate W <- P(W) from W = G (= P(top)) until a fixed point."""
    cache = _vals(prob)
    G, g, rows, avoid = cache
    W = [INF if avoid[x] else G[x] for x in range(prob.n)]
    limit = max_iter if max_iter is not None else 4 * prob.n + 8
    for it in range(limit):
        N = apply_P(prob, W, cache)
        if N == W:
            return W, it
        W = N
    raise Diverged()


def evaluate(prob, choice):
    """L(., mu) for the deterministic controller `choice[x]` in
    {-1 (hand over), -2 (none), 0..K-1}."""
    G, g, rows, avoid = _vals(prob)
    K = prob.K
    W = [INF if avoid[x] else G[x] for x in range(prob.n)]
    for _ in range(4 * prob.n + 8):
        N = []
        for x in range(prob.n):
            c = choice[x]
            if avoid[x] or c == -2:
                N.append(INF)
            elif c == -1:
                N.append(G[x])
            else:
                p = x * K + c
                N.append(min(G[x], max(g[p] + h + W[y] for y, h in rows[p])))
        if N == W:
            return W
        W = N
    raise Diverged()


def enumerate_V(prob):
    """Pointwise minimum of L(., mu) over all deterministic memoryless
    controllers mu: X -> U (hand-over at any time is part of L's inf over v).
    Controllers whose closed loop diverges contribute -inf."""
    n, K = prob.n, prob.K
    best = [INF] * n
    for choice in itertools.product(range(K), repeat=n):
        try:
            L = evaluate(prob, list(choice))
        except Diverged:
            L = [-INF] * n
        best = [min(a, b) for a, b in zip(best, L)]
    return best


def cost_J(prob, u_sig, v_sig, x_sig, cost_of=None):
    """J(u,v,x) = G(x(T)) + sum_{t<T} g(x(t), x(t+1), u(t)), T = first t with
    v(t) = 1; INF if v never switches.  `cost_of(x, y, u)` defaults to the
    problem's running cost g(x,u) + h(x,y,u)."""
    G, g, rows, avoid = _vals(prob)
    K = prob.K
    if 1 not in v_sig:
        return INF
    T = v_sig.index(1)
    tot = G[x_sig[T]]
    for t in range(T):
        p = x_sig[t] * K + u_sig[t]
        hy = dict(rows[p])
        assert x_sig[t + 1] in hy, "not a behavior of the system"
        tot += cost_of(x_sig[t], x_sig[t + 1], u_sig[t]) if cost_of else g[p] + hy[x_sig[t + 1]]
    return tot


def kleene_np(prob, dtype=np.float64, max_iter=100000):
    """Vectorised Kleene iteration W <- P(W) from G over CSR rows.

    Values are carried as `dtype` floats (+inf = INF); int32 problems are
    evaluated exactly in float64 (all sums stay far below 2^53).  float32 uses
    one single-precision addition per backup."""
    n, K = prob.n, prob.K
    ptr = np.asarray(prob.succ_ptr, dtype=np.int64)
    idx = np.asarray(prob.succ_idx, dtype=np.int64)
    if prob.dtype == "i32":
        G = np.where(prob.G >= INF_I32, np.inf, prob.G.astype(np.float64)).astype(dtype)
        g = np.where(prob.g >= INF_I32, np.inf, prob.g.astype(np.float64)).astype(dtype)
    else:
        G = prob.G.astype(dtype)
        g = prob.g.astype(dtype)
    he = getattr(prob, "g_edge", None)
    h = None if he is None else np.asarray(he, dtype=np.float64 if prob.dtype == "i32" else np.float32).astype(dtype)
    av = prob.avoid.astype(bool)
    W = np.where(av, np.inf, G).astype(dtype)
    starts = ptr[:-1]
    for it in range(max_iter):
        Wy = W[idx] if h is None else (h + W[idx]).astype(dtype)
        mx = np.maximum.reduceat(Wy, starts)
        d = (g + mx).astype(dtype)
        best = d.reshape(n, K).min(axis=1)
        N = np.minimum(G, best).astype(dtype)
        N[av] = np.inf
        if np.array_equal(N, W):
            if prob.dtype == "i32":
                out = np.where(np.isinf(W), INF_I32, W).astype(np.int64)
                return out.astype(np.int32), it
            return W, it
        if it > 4 * n + 8:
            raise Diverged()
        W = N
    raise Diverged()
