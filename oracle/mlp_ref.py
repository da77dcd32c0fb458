"""fp64 reference of the frontier-ordering network — TEST INFRASTRUCTURE ONLY.

The network orders the solver's frontier; it never touches the values it
computes.  A small multilayer perceptron 4 -> 64 -> 64 -> 1 with ReLU maps
normalised cell coordinates (relative to the centre of the target) to a
prediction of V / scale.  Its weights are stored in bfloat16 (a working
copy, rounded to nearest even from an fp32 master copy); the library
computes with them in fp32.  This module does the same arithmetic in fp64
from the same bf16 weights, with plain matrix products, and differentiates
it by hand:

  forward   a1 = W1 f + b1, h1 = relu(a1), a2 = W2 h1 + b2, h2 = relu(a2),
            out = W3 . h2 + b3
  loss      mean of (out - y)^2 over the samples with a finite label y
  gradient  chain rule through the three layers (ReLU'(0) = 0)
  Adam      Kingma & Ba (2015): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
            theta <- theta - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
  keys      vhat = scale * out, key = clamp(floor((vhat - min vhat) / width),
            0, 65535) as a 16-bit bucket index

The keys are evaluated for every cell of an instance; there the library
feeds h1 to the second layer as two bfloat16 terms (hi + lo, products with
the bf16 weights summed in fp32: the matrix-core form of an fp32 product).
split_hidden_error_bound bounds how far that evaluation may land from the
fp64 forward pass.

Parameter vector layout (4545 values): W1 [64][4] row-major, b1 [64],
W2 [64][64] row-major (W2[j][k] multiplies h1[k] into unit j), b2 [64],
W3 [64], b3 [1].

Pins (tests/test_oracle_mlp.py): bf16 rounding against hand-worked ties and
torch's conversion; the two-term bf16 split against hand-worked values and
its bound against an emulated fp32 evaluation; the forward pass against a hand-built network with a
closed-form output and against torch.nn.functional in fp64; the gradient
against central finite differences and against torch.autograd; Adam
against its closed-form first step and torch.optim.Adam; the features and
keys against hand-computed values.
"""
from __future__ import annotations

import numpy as np

H = 64
NIN = 4
SIZES = (("W1", (H, NIN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,)))
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 4545
OFFSETS = {}
_o = 0
for _name, _shape in SIZES:
    OFFSETS[_name] = (_o, _shape)
    _o += int(np.prod(_shape))


def bf16_round(x) -> np.ndarray:
    """Round fp32 values to the nearest bfloat16, ties to even; returned as
    float32 (every bf16 value is exactly representable in fp32)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).copy()
    out[nan] = np.float32("nan")
    return out


def bf16_bits(x) -> np.ndarray:
    """The 16-bit patterns of bf16_round(x)."""
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def unpack(theta):
    """Views of the parameter vector as (W1, b1, W2, b2, W3, b3)."""
    t = np.asarray(theta, dtype=np.float64)
    assert t.shape == (NPARAMS,)
    return tuple(t[o:o + int(np.prod(s))].reshape(s) for o, s in (OFFSETS[n] for n, _ in SIZES))


def features(cells, dims, tcx, tcy) -> np.ndarray:
    """Normalised cell-centre coordinates, the first two relative to the
    target centre (tcx, tcy): ((x0+.5-tcx)/N0, (x1+.5-tcy)/N1, (x2+.5)/N2,
    (x3+.5)/N3), with x = x0 + N0*(x1 + N1*(x2 + N2*x3))."""
    c = np.asarray(cells, dtype=np.int64)
    N = [int(d) for d in dims]
    x0 = c % N[0]
    r = c // N[0]
    x1 = r % N[1]
    r //= N[1]
    x2 = r % N[2]
    x3 = r // N[2]
    f = np.empty((c.size, NIN), dtype=np.float64)
    f[:, 0] = (x0 + 0.5 - float(tcx)) / N[0]
    f[:, 1] = (x1 + 0.5 - float(tcy)) / N[1]
    f[:, 2] = (x2 + 0.5) / N[2]
    f[:, 3] = (x3 + 0.5) / N[3]
    return f


def forward(theta_bf16, F):
    """Network output for each row of F, plus the pre-activations."""
    W1, b1, W2, b2, W3, b3 = unpack(theta_bf16)
    F = np.asarray(F, dtype=np.float64)
    a1 = F @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    out = h2 @ W3 + b3[0]
    return out, (F, a1, h1, a2, h2)


def loss_grad(theta_bf16, F, y):
    """Mean squared error over the finite labels and its gradient with
    respect to the (bf16) parameters.  Returns (loss, grad[4545], count)."""
    y = np.asarray(y, dtype=np.float64)
    out, (F, a1, h1, a2, h2) = forward(theta_bf16, F)
    W1, b1, W2, b2, W3, b3 = unpack(theta_bf16)
    fin = np.isfinite(y)
    cnt = int(fin.sum())
    g = np.zeros(NPARAMS)
    if cnt == 0:
        return 0.0, g, 0
    r = np.where(fin, out - np.where(fin, y, 0.0), 0.0)
    loss = float((r * r).sum() / cnt)
    dout = 2.0 * r / cnt                      # d loss / d out
    dW3 = h2.T @ dout
    db3 = dout.sum()
    da2 = np.outer(dout, W3) * (a2 > 0)       # through relu
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * (a1 > 0)
    dW1 = da1.T @ F
    db1 = da1.sum(axis=0)
    parts = {"W1": dW1, "b1": db1, "W2": dW2, "b2": db2, "W3": dW3, "b3": np.array([db3])}
    for name, _ in SIZES:
        o, s = OFFSETS[name]
        g[o:o + int(np.prod(s))] = parts[name].reshape(-1)
    return loss, g, cnt


ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_step(master, m, v, t, grad, lr):
    """One Adam update (step number t >= 1) of the fp32 master weights.
    Returns (master, m, v) in fp64."""
    m = ADAM_B1 * np.asarray(m, np.float64) + (1 - ADAM_B1) * grad
    v = ADAM_B2 * np.asarray(v, np.float64) + (1 - ADAM_B2) * grad * grad
    mh = m / (1 - ADAM_B1 ** t)
    vh = v / (1 - ADAM_B2 ** t)
    master = np.asarray(master, np.float64) - lr * mh / (np.sqrt(vh) + ADAM_EPS)
    return master, m, v


def vhat(theta_bf16, F, scale=1000.0):
    out, _ = forward(theta_bf16, F)
    return scale * out


def keys_from_vhat(vh, width=16.0):
    """Bucket keys: floor((vhat - min vhat) / width) clamped to [0, 65535]."""
    vh = np.asarray(vh, dtype=np.float64)
    k = np.floor((vh - vh.min()) / float(width))
    return np.clip(k, 0, 65535).astype(np.uint16)


def out_error_bound(theta_bf16, F):
    """A bound on |fl32(out) - out| for the fp32 evaluation (sequential fused
    multiply-adds per unit, features rounded once): with u = 2^-24 and the
    same network applied to absolute values (|W|, |b|, |f|), every sum of
    length L contributes at most L*u times its absolute magnitude, and the
    layer errors propagate through |W|.  A generous factor 2 covers the
    second-order terms."""
    W1, b1, W2, b2, W3, b3 = unpack(theta_bf16)
    u = 2.0 ** -24
    F = np.abs(np.asarray(F, dtype=np.float64))
    m1 = F @ np.abs(W1).T + np.abs(b1)             # |a1| magnitude
    e1 = (NIN + 2) * u * m1                         # features + 4 fma + bias
    m2 = m1 @ np.abs(W2).T + np.abs(b2)
    e2 = (H + 1) * u * m2 + e1 @ np.abs(W2).T
    m3 = m2 @ np.abs(W3) + abs(b3[0])
    e3 = (H + 1) * u * m3 + e2 @ np.abs(W3)
    return 2.0 * e3



def split_hidden_error_bound(theta_bf16, F):
    """A bound on |library out - forward out| per row of F for the per-cell
    key evaluation, which works as follows: each feature takes two fp32
    roundings (a subtraction and a division); a1 is formed from them in fp32
    in any order (4 products and 5 additions, each rounded at most once);
    h1 = relu(a1) enters the second layer as two bf16 terms hi = bf16(h1),
    lo = bf16(h1 - hi), whose products with the bf16 weights are exact and
    are summed with b2 in fp32 in any order; the third layer is fp32 in any
    order.

    With u = 2^-24, exact activations h1, h2 (fp64 forward pass) and |.| of
    weights taken elementwise:
      a1:  within e1 = 3 NIN u (|F| |W1|^T + |b1|) (11 u to first order);
      h1:  relu is 1-Lipschitz and |h1 - hi - lo| <= 2^-16 |h1| (hi is h1 to
           8 significant bits, lo the rest to 8 more), so hi + lo is within
           eh = e1 + 2^-16 (h1 + e1) of the exact h1;
      a2:  2H + 1 fp32 additions of terms whose absolute sum is at most
           m2 = (1 + 2^-8) |W2| (h1 + e1) + |b2|: e2 = (2H + 2) u m2 + |W2| eh;
      out: m3 = |W3| (h2 + e2) + |b3|: e3 = (H + 2) u m3 + |W3| e2.
    A factor 2 covers the second-order terms."""
    W1, b1, W2, b2, W3, b3 = unpack(theta_bf16)
    u = 2.0 ** -24
    F = np.asarray(F, dtype=np.float64)
    _, (_, a1, h1, a2, h2) = forward(theta_bf16, F)
    e1 = 3 * NIN * u * (np.abs(F) @ np.abs(W1).T + np.abs(b1))
    eh = e1 + 2.0 ** -16 * (h1 + e1)
    m2 = (1 + 2.0 ** -8) * ((h1 + e1) @ np.abs(W2).T) + np.abs(b2)
    e2 = (2 * H + 2) * u * m2 + eh @ np.abs(W2).T
    m3 = (h2 + e2) @ np.abs(W3) + abs(b3[0])
    e3 = (H + 2) * u * m3 + e2 @ np.abs(W3)
    return 2.0 * e3
