"""GPU parity of the frontier-ordering network against its fp64 reference
(oracle/mlp_ref.py): bf16 rounding, features, forward pass, gradient, Adam
steps and bucket keys; and the bucket-ordered solve driven by the network's
keys, bit-exact with the oracle.

Tolerances come from the arithmetic: the library evaluates the network in
fp32 with fused multiply-adds from the same bf16 weights, so its outputs lie
within mlp_ref.out_error_bound of the fp64 values; gradients are sums of
such products over the minibatch (relative L2 error of a few fp32 ulps of
the summed magnitudes, bounded here by 1e-4); a bucket key is compared
wherever the reference quotient (vhat - min) / width is farther than its
error bound from an integer."""
import numpy as np
import pytest

import oracle
import paper_2001_06231_amd as gbf
import synth
from oracle import mlp_ref as M
from paper_2001_06231_amd import learn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    gbf.lib()


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _params(seed, scale=None):
    if scale is None:
        return learn.init_params(seed)
    return ((synth.Stream(seed, 9).uniform(M.NPARAMS) * 2 - 1) * scale).astype(np.float32)


def _feats(seed, n):
    return ((synth.Stream(seed, 2).uniform(n * 4) * 2 - 1).reshape(n, 4)).astype(np.float32)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_bf16_working_copy():
    _case("mlp bf16 rounding")
    vals = np.zeros(M.NPARAMS, np.float32)
    special = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-8 + 2**-20, -2.5, 3e38, -1e-30, 65504.0],
                       dtype=np.float32)
    vals[:special.size] = special
    vals[special.size:] = (synth.Stream(3, 3).uniform(M.NPARAMS - special.size).astype(np.float32) - 0.5) * 7
    net = gbf.MLP(vals)
    master, bf = net.params()
    assert np.array_equal(master, vals)
    assert np.array_equal(bf, M.bf16_bits(vals))
    net.free()


def test_samples_features_and_labels():
    _case("mlp samples")
    import torch
    dims = (13, 11, 7, 5)
    n = int(np.prod(dims))
    V = (synth.Stream(4, 4).raw(n) % np.uint64(5000)).astype(np.int32)
    V[::17] = synth.INF_I32
    cells = (synth.Stream(5, 5).raw(3000) % np.uint64(n)).astype(np.int64)
    cells[7] = n + 3   # outside the grid
    cells[8] = -1
    net = gbf.MLP(learn.init_params(1))
    f, t = net.samples(dims, (4.5, 2.25), _dev(cells), V=_dev(V), scale=1000.0)
    f, t = f.cpu().numpy(), t.cpu().numpy()
    ok = (cells >= 0) & (cells < n)
    ref = M.features(cells[ok], dims, 4.5, 2.25)
    assert np.allclose(f[ok], ref, rtol=4e-7, atol=4e-7)
    assert np.isnan(f[~ok]).all() and np.isnan(t[~ok]).all()
    lab = V[cells[ok]].astype(np.float64)
    want = np.where(lab == synth.INF_I32, np.nan, lab / 1000.0)
    assert np.array_equal(np.isnan(t[ok]), np.isnan(want))
    fin = ~np.isnan(want)
    assert np.allclose(t[ok][fin], want[fin], rtol=1.2e-7, atol=0)
    # fp32 values: INF -> no label
    Vf = np.where(V == synth.INF_I32, np.inf, V.astype(np.float32) * 0.5).astype(np.float32)
    _, tf = net.samples(dims, (4.5, 2.25), _dev(cells), V=_dev(Vf), scale=1000.0)
    tf = tf.cpu().numpy()
    assert np.array_equal(np.isnan(tf[ok]), np.isinf(Vf[cells[ok]]))
    net.free()
    del torch


@pytest.mark.parametrize("count", [1, 63, 64, 1000, 4099])
def test_forward(count):
    _case(f"mlp forward {count}")
    p = _params(7)
    net = gbf.MLP(p)
    F = _feats(8, count)
    out = net.forward(_dev(F)).cpu().numpy().astype(np.float64)
    th = M.bf16_round(p).astype(np.float64)
    ref, _ = M.forward(th, F.astype(np.float64))
    bound = M.out_error_bound(th, F.astype(np.float64))
    assert (np.abs(out - ref) <= bound).all(), np.max(np.abs(out - ref) / bound)
    net.free()


@pytest.mark.parametrize("count,with_idx", [(1, False), (64, False), (1000, True), (4099, True)])
def test_gradient_matches_oracle(count, with_idx):
    _case(f"mlp gradient {count} idx={with_idx}")
    p = _params(11, scale=0.3)
    net = gbf.MLP(p)
    rows = count + 37
    F = _feats(12, rows)
    y = (synth.Stream(13, 3).uniform(rows) * 2 - 0.5).astype(np.float32)
    y[::5] = np.nan
    if with_idx:
        idx = (synth.Stream(14, 4).raw(count) % np.uint64(rows)).astype(np.int64)
        g, loss, lab = net.grad(_dev(F), _dev(y), _dev(idx))
        Fs, ys = F[idx], y[idx]
    else:
        g, loss, lab = net.grad(_dev(F[:count]), _dev(y[:count]))
        Fs, ys = F[:count], y[:count]
    th = M.bf16_round(p).astype(np.float64)
    rl, rg, rc = M.loss_grad(th, Fs.astype(np.float64), ys.astype(np.float64))
    assert lab == rc
    if rc == 0:
        assert loss == 0 and not g.any()
        return
    assert abs(loss - rl) <= 1e-5 * max(rl, 1e-6)
    err = np.linalg.norm(g.astype(np.float64) - rg) / np.linalg.norm(rg)
    assert err <= 1e-4, err
    net.free()


def test_gradient_skips_bad_indices():
    _case("mlp gradient bad indices")
    p = _params(15, scale=0.3)
    net = gbf.MLP(p)
    F = _feats(16, 100)
    y = synth.Stream(17, 3).uniform(100).astype(np.float32)
    idx = np.arange(100, dtype=np.int64)
    idx[10] = 100   # outside the rows
    idx[20] = -5
    g, loss, lab = net.grad(_dev(F), _dev(y), _dev(idx))
    keep = np.array([i for i in range(100) if i not in (10, 20)])
    th = M.bf16_round(p).astype(np.float64)
    rl, rg, rc = M.loss_grad(th, F[keep].astype(np.float64), y[keep].astype(np.float64))
    assert lab == rc == 98
    assert np.linalg.norm(g - rg) <= 1e-4 * np.linalg.norm(rg)
    net.free()


def test_adam_steps_match_oracle():
    """Twenty Adam steps on a fixed minibatch: the fp32 master weights track
    the fp64 reference trajectory, the working copy is the bf16 rounding of
    the master, and the loss falls."""
    _case("mlp adam")
    p = learn.init_params(21)
    net = gbf.MLP(p)
    F = _feats(22, 512)
    y = (0.3 * F[:, 0] - 0.2 * F[:, 1] + 0.1).astype(np.float32)
    Fd, yd = _dev(F), _dev(y)
    master = p.astype(np.float64)
    m = np.zeros(M.NPARAMS)
    v = np.zeros(M.NPARAMS)
    losses = []
    for t in range(1, 21):
        lg = net.train_step(Fd, yd, lr=1e-3, want_loss=True)
        th = M.bf16_round(master.astype(np.float32)).astype(np.float64)
        rl, rg, _ = M.loss_grad(th, F.astype(np.float64), y.astype(np.float64))
        assert abs(lg - rl) <= 1e-4 * rl + 1e-7, (t, lg, rl)
        losses.append(rl)
        master, m, v = M.adam_step(master, m, v, t, rg, 1e-3)
        gm, gb = net.params()
        # a step moves a weight by about lr: differences in the gradient
        # show up as a small fraction of it
        assert np.max(np.abs(gm - master)) <= 2e-5 * t, (t, np.max(np.abs(gm - master)))
        assert np.array_equal(gb, M.bf16_bits(gm))
    assert losses[-1] < losses[0]
    net.free()


@pytest.mark.parametrize("dims,width", [((30, 20, 6, 4), 16.0), ((9, 7, 3, 2), 1.0), ((64, 1, 1, 1), 16.0)])
def test_bucket_keys(dims, width):
    _case(f"mlp keys {dims}")
    import torch
    p = learn.init_params(31)
    net = gbf.MLP(p)
    n = int(np.prod(dims))
    tc = (dims[0] / 2 - 0.5, dims[1] / 3)
    vhat = torch.empty(n, dtype=torch.float32, device="cuda")
    keys, vmin = net.bucket_keys(dims, tc, scale=1000.0, width=width, vhat=vhat)
    keys = keys.cpu().numpy().view(np.uint16)
    vh = vhat.cpu().numpy().astype(np.float64)
    th = M.bf16_round(p).astype(np.float64)
    F = M.features(np.arange(n), dims, np.float32(tc[0]), np.float32(tc[1]))
    # the key kernel feeds h1 to the matrix cores as two bf16 terms
    ref = M.vhat(th, F, 1000.0)
    tol = 1000.0 * M.split_hidden_error_bound(th, F) * 1.0001 + 1e-3
    assert (np.abs(vh - ref) <= tol).all()
    # the minimum and the keys are decided in fp32 from the kernel's values
    v32 = vhat.cpu().numpy()
    assert np.float32(vmin) == v32.min()
    q = np.floor((v32 - np.float32(vmin)) / np.float32(width))
    assert np.array_equal(keys, np.clip(q, 0, 65535).astype(np.uint16))
    # the keys equal the reference's except where a value lies within the
    # kernel's rounding error of a bucket edge
    agree = float((keys == M.keys_from_vhat(ref, width)).mean())
    err = np.abs(vh - ref)
    print(f"keys equal to the reference's: {agree:.5f}; |vhat - ref| max {err.max():.3g}, "
          f"bound max {tol.max():.3g}", flush=True)
    if width >= 16:
        assert agree > 0.99
    net.free()


def test_learned_keys_drive_exact_solve():
    """Keys from the network (trained for a few steps on this instance's own
    values) order a bucketed solve whose values and policy equal the
    oracle's."""
    _case("mlp keys -> bucketed solve")
    import torch
    prob = synth.grid4d(synth.instance_seed(53, 0), dims=(18, 16, 10, 6), K=16)
    ref = oracle.solve(prob)
    net = gbf.MLP(learn.init_params(41))
    g = gbf.load_problem(prob, encoding="csr")
    V = torch.empty(prob.n, dtype=torch.int32, device="cuda")
    g.solve(V)
    cells = _dev(np.arange(prob.n, dtype=np.int64))
    tc = learn.target_centre(prob)
    f, t = net.samples(prob.dims, tc, cells, V=V, scale=1000.0)
    for _ in range(50):
        net.train_step(f, t, lr=3e-3)
    keys, _ = net.bucket_keys(prob.dims, tc, scale=1000.0, width=16.0)
    status, st, Vb = g.solve(order="buckets", bucket_key=keys)
    pol, res = g.policy()
    # a briefly trained network may exceed the plain solve's work; the
    # solve then finishes in plain order (fallback 1), still exact
    assert status == gbf.OK and st["fallback"] in (0, 1) and res == 0
    assert np.array_equal(Vb, ref["V"])
    assert np.array_equal(pol, ref["policy"])
    _, st_p, _ = g.solve(order="plain")
    print(f"pair evaluations: learned buckets {st['pair_evals']} plain {st_p['pair_evals']}; "
          f"rounds {st['rounds']} vs {st_p['rounds']}", flush=True)
    g.free()
    net.free()


@pytest.mark.timeout(600)
def test_learned_order_full_size():
    """The learned-ordering workload at full size (60x60x30x12, 16 inputs,
    1.296 M cells; held-out instance 1000) with the trained weights and the
    default bucket window: values and policy equal the oracle's everywhere,
    and the relaxation count is below the plain order's."""
    _case("learned order, full size")
    import torch
    prob = synth.learned_instance(1000, with_csr=False)
    ref = oracle.solve(prob)
    print("oracle done", flush=True)
    net = gbf.MLP(learn.load_params())
    g = gbf.load_problem(prob, encoding="csr")
    keys, _ = net.bucket_keys(prob.dims, learn.target_centre(prob), learn.SCALE, learn.WIDTH)
    V = torch.empty(prob.n, dtype=torch.int32, device="cuda")
    status, st, _ = g.solve(V, order="buckets", bucket_key=keys)
    pol, res = g.policy()
    assert status == gbf.OK and st["fallback"] == 0 and res == 0
    Vh = V.cpu().numpy()
    bad = np.nonzero(Vh != ref["V"])[0]
    assert bad.size == 0, (bad[:8], Vh[bad[:8]], ref["V"][bad[:8]])
    assert np.array_equal(pol, ref["policy"])
    _, st_p, _ = g.solve(V)
    print(f"edge relaxations: learned {st['edge_relax']} plain {st_p['edge_relax']}", flush=True)
    assert st["edge_relax"] < st_p["edge_relax"]
    g.free()
    net.free()
