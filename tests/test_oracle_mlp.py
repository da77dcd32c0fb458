"""Pins of the fp64 network reference (oracle/mlp_ref.py) against things
other than itself: hand-worked bf16 ties, a network with a closed-form
output, finite differences, torch's own fp64 autograd and Adam, and
hand-computed features and keys."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp_ref as M


def _theta(seed, scale=0.3):
    s = synth.Stream(seed, 1)
    return M.bf16_round((s.uniform(M.NPARAMS) * 2 - 1) * scale).astype(np.float64)


def _feats(seed, n):
    s = synth.Stream(seed, 2)
    return (s.uniform(n * 4).reshape(n, 4) * 2 - 1)


def test_layout():
    assert M.NPARAMS == 4545
    assert M.OFFSETS["W2"] == (320, (64, 64))
    assert M.OFFSETS["b3"] == (4544, (1,))


def test_bf16_ties_and_library():
    one = np.float32(1.0)
    cases = {
        1.0: 1.0,
        1.0 + 2.0 ** -8: 1.0,                          # tie -> even (1.0)
        1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,          # tie -> even (mantissa ...10)
        1.0 + 2.0 ** -8 + 2.0 ** -20: 1.0 + 2.0 ** -7,  # above the tie
        -2.5: -2.5,
        3.0e38: 226 / 128 * 2.0 ** 127,                 # 1.7632 -> 226/128 (big values stay finite)
    }
    for x, want in cases.items():
        got = float(M.bf16_round(np.float32(x)).reshape(-1)[0])
        assert got == want, (x, got, want)
    assert np.isnan(M.bf16_round(np.float32("nan")))
    xs = (synth.Stream(5, 5).uniform(10000).astype(np.float32) - 0.5) * np.float32(1e3)
    lib = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(M.bf16_round(xs), lib)
    assert float(one) == 1.0
    bits = M.bf16_bits(np.array([1.0, -2.0], np.float32))
    assert list(bits) == [0x3F80, 0xC000]


def test_forward_closed_form():
    """W1 routes feature i to unit i (i < 4), W2 is the identity, W3 sums:
    out = sum_i relu(f_i) + b3."""
    th = np.zeros(M.NPARAMS)
    W1, b1, W2, b2, W3, b3 = M.unpack(th)  # views into th
    for i in range(4):
        W1[i, i] = 1.0
    W2[:] = np.eye(64)
    W3[:] = 1.0
    b3[0] = 0.25
    F = _feats(11, 50)
    out, _ = M.forward(th, F)
    assert np.allclose(out, np.maximum(F, 0).sum(axis=1) + 0.25, rtol=0, atol=1e-15)


def _torch_net(theta):
    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    W1 = t[0:256].view(64, 4)
    b1 = t[256:320]
    W2 = t[320:4416].view(64, 64)
    b2 = t[4416:4480]
    W3 = t[4480:4544]
    b3 = t[4544]

    def f(F):
        h1 = torch.nn.functional.relu(torch.nn.functional.linear(F, W1, b1))
        h2 = torch.nn.functional.relu(torch.nn.functional.linear(h1, W2, b2))
        return h2 @ W3 + b3
    return t, f


def test_forward_and_grad_match_torch_autograd():
    th = _theta(21)
    F = _feats(22, 300)
    y = synth.Stream(23, 3).uniform(300) * 2
    y[::7] = np.nan  # unlabelled samples are skipped
    loss, g, cnt = M.loss_grad(th, F, y)
    assert cnt == 300 - len(range(0, 300, 7))
    t, net = _torch_net(th)
    Ft = torch.tensor(F)
    out = net(Ft)
    ref_out, _ = M.forward(th, F)
    assert np.allclose(out.detach().numpy(), ref_out, rtol=1e-13, atol=1e-13)
    fin = torch.tensor(np.isfinite(y))
    yt = torch.tensor(np.nan_to_num(y))
    lt = ((out - yt)[fin] ** 2).mean()
    lt.backward()
    assert abs(float(lt.detach()) - loss) <= 1e-12 * max(1.0, loss)
    gt = t.grad.numpy()
    assert np.linalg.norm(g - gt) <= 1e-11 * np.linalg.norm(gt)


def test_grad_finite_differences():
    th = _theta(31)
    F = _feats(32, 64)
    y = synth.Stream(33, 3).uniform(64)
    _, g, _ = M.loss_grad(th, F, y)
    out, (_, a1, _, a2, _) = M.forward(th, F)
    h = 1e-6
    s = synth.Stream(34, 4)
    idx = (s.raw(60) % np.uint64(M.NPARAMS)).astype(np.int64)
    checked = 0
    for i in idx:
        tp = th.copy()
        tm = th.copy()
        tp[i] += h
        tm[i] -= h
        # skip coordinates whose step crosses a ReLU kink
        _, (_, a1p, _, a2p, _) = M.forward(tp, F)
        _, (_, a1m, _, a2m, _) = M.forward(tm, F)
        if ((a1p > 0) != (a1m > 0)).any() or ((a2p > 0) != (a2m > 0)).any():
            continue
        fd = (M.loss_grad(tp, F, y)[0] - M.loss_grad(tm, F, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])), (i, fd, g[i])
        checked += 1
    assert checked > 30


def test_adam_first_step_closed_form():
    grad = np.array([0.5, -2.0, 1e-3, 0.0])
    master = np.array([1.0, 1.0, 1.0, 1.0])
    new, m, v = M.adam_step(master, np.zeros(4), np.zeros(4), 1, grad, 1e-3)
    # m_hat = g, v_hat = g^2: the first step is lr * g / (|g| + eps)
    want = master - 1e-3 * grad / (np.abs(grad) + M.ADAM_EPS)
    assert np.allclose(new, want, rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * grad) and np.allclose(v, 0.001 * grad * grad)


def test_adam_matches_torch():
    th = _theta(41)
    grads = [(synth.Stream(42 + k, 5).uniform(M.NPARAMS) - 0.5) for k in range(5)]
    p = torch.tensor(th.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(M.ADAM_B1, M.ADAM_B2), eps=M.ADAM_EPS)
    master, m, v = th.copy(), np.zeros(M.NPARAMS), np.zeros(M.NPARAMS)
    for t, gk in enumerate(grads, start=1):
        opt.zero_grad()
        p.grad = torch.tensor(gk)
        opt.step()
        master, m, v = M.adam_step(master, m, v, t, gk, 1e-3)
    assert np.allclose(master, p.detach().numpy(), rtol=0, atol=1e-14)


def test_features_by_hand():
    dims = (4, 3, 2, 2)
    # cell 0 = (0,0,0,0); cell 4*3*2 + 4*3 + 4 + 3 = (3,1,1,1)
    f = M.features([0, 24 + 12 + 4 + 3], dims, tcx=1.5, tcy=0.5)
    assert np.allclose(f[0], [(0.5 - 1.5) / 4, (0.5 - 0.5) / 3, 0.5 / 2, 0.5 / 2])
    assert np.allclose(f[1], [(3.5 - 1.5) / 4, (1.5 - 0.5) / 3, 1.5 / 2, 1.5 / 2])


def test_keys_by_hand():
    vh = np.array([100.0, 115.9, 116.0, 131.99, 1e9, 99.5])
    k = M.keys_from_vhat(vh, 16.0)
    assert list(k) == [0, 1, 1, 2, 65535, 0]


def test_error_bound_covers_fp32_evaluation():
    """The bound holds for a plain fp32 evaluation of the same network (numpy
    float32 products, one rounding per operation)."""
    th = M.bf16_round(_theta(51, scale=0.5)).astype(np.float64)
    F = _feats(52, 500)
    out, _ = M.forward(th, F)
    W1, b1, W2, b2, W3, b3 = (a.astype(np.float32) for a in M.unpack(th))
    F32 = F.astype(np.float32)
    h1 = np.zeros((500, 64), np.float32)
    for j in range(64):
        acc = b1[j] + np.zeros(500, np.float32)
        for i in range(4):
            acc = acc + W1[j, i] * F32[:, i]
        h1[:, j] = np.maximum(acc, 0)
    h2 = np.zeros((500, 64), np.float32)
    for j in range(64):
        acc = b2[j] + np.zeros(500, np.float32)
        for k in range(64):
            acc = acc + W2[j, k] * h1[:, k]
        h2[:, j] = np.maximum(acc, 0)
    o = b3[0] + np.zeros(500, np.float32)
    for j in range(64):
        o = o + W3[j] * h2[:, j]
    err = np.abs(o.astype(np.float64) - out)
    bound = M.out_error_bound(th, F)
    # products are rounded separately here (no fma): add one u per term
    assert (err <= 2 * bound).all()


def test_split_by_hand():
    """hi = bf16(h), lo = bf16(h - hi): hand-worked values, and the residual
    bound |h - hi - lo| <= 2^-16 |h| on many values."""
    def split(h):
        h = np.float32(h)
        hi = M.bf16_round(h).reshape(-1)[0]
        lo = M.bf16_round(np.float32(h - hi)).reshape(-1)[0]
        return float(hi), float(lo)
    # 1 + 2^-8 + 2^-20: hi rounds up to 1 + 2^-7; the rest, -(2^-8 - 2^-20),
    # has 12 significant bits and rounds to -2^-8
    assert split(1.0 + 2.0 ** -8 + 2.0 ** -20) == (1.0 + 2.0 ** -7, -(2.0 ** -8))
    # 3 + 2^-10: hi = 3 (the tail is below half a bf16 step), lo = 2^-10 exactly
    assert split(3.0 + 2.0 ** -10) == (3.0, 2.0 ** -10)
    # a bf16 value splits into itself and zero
    assert split(-2.5) == (-2.5, 0.0)
    h = (synth.Stream(91, 1).uniform(20000).astype(np.float32) * np.float32(50))
    hi = M.bf16_round(h)
    lo = M.bf16_round((h - hi).astype(np.float32))
    r = np.abs(h.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert (r <= 2.0 ** -16 * np.abs(h.astype(np.float64))).all()
    assert r.max() > 2.0 ** -19 * np.abs(h).max()   # and is not far from tight


def test_split_bound_covers_fp32_evaluation():
    """The bound holds for an evaluation in the key kernel's shape: fp32
    features, a1 by fused multiply-adds (emulated: the exact fp64
    product-sum rounded to fp32 once per step), relu, the two-term bf16
    split, fp32 pairwise sums of the exact products of the later layers."""
    th = M.bf16_round(_theta(81, scale=0.5)).astype(np.float64)
    n = 3000
    F = _feats(82, n)
    F32 = F.astype(np.float32).astype(np.float64)
    out, _ = M.forward(th, F)
    W1, b1, W2, b2, W3, b3 = M.unpack(th)
    a1 = np.tile(b1.astype(np.float32).astype(np.float64), (n, 1))
    for i in range(4):
        a1 = (a1 + F32[:, i:i + 1] * W1[:, i]).astype(np.float32).astype(np.float64)
    h1 = np.maximum(a1, 0).astype(np.float32)
    hi = M.bf16_round(h1)
    lo = M.bf16_round((h1 - hi).astype(np.float32))

    def sum32(terms):   # pairwise fp32 sum along the last axis
        t = terms.astype(np.float32)
        while t.shape[-1] > 1:
            t = (t[..., 0::2] + t[..., 1::2]).astype(np.float32)
        return t[..., 0].astype(np.float64)

    prods = np.concatenate([hi.astype(np.float64)[:, None, :] * W2[None, :, :],
                            lo.astype(np.float64)[:, None, :] * W2[None, :, :]], axis=2)
    a2 = (sum32(prods) + b2).astype(np.float32).astype(np.float64)
    h2 = np.maximum(a2, 0)
    o = (sum32(h2 * W3) + b3[0]).astype(np.float32).astype(np.float64)
    err = np.abs(o - out)
    bound = M.split_hidden_error_bound(th, F)
    assert (err <= bound).all()
    # the bound is far below the output scale, for every row, and below
    # what a single bf16 rounding of h1 would cost on many rows
    assert bound.max() < 5e-3 * np.abs(out).max()
    # and the split evaluation is much closer than a single bf16 rounding of h1
    h1b = hi.astype(np.float64)
    o1 = np.maximum(h1b @ W2.T + b2, 0) @ W3 + b3[0]
    assert err.max() < 0.05 * np.abs(o1 - out).max()
    assert (np.abs(o1 - out) > bound).mean() > 0.1


@pytest.mark.parametrize("n", [1, 5])
def test_loss_grad_no_labels(n):
    th = _theta(61)
    F = _feats(62, n)
    loss, g, cnt = M.loss_grad(th, F, np.full(n, np.nan))
    assert cnt == 0 and loss == 0.0 and not g.any()
