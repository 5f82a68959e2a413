"""GPU parity of the learned-closure kernels against the FP64 closure oracle.

Bars: the BF16 matrix-core forward within 5e-4 relative (Frobenius) of the
oracle that rounds at the same storage points, and within 2e-2 of the oracle
that rounds only inputs and weights; weight gradients within 1e-3 (same
rounding points) and 1e-2 (inputs and weights rounded only) relative
(Frobenius) per tensor; the loss gradient, Adam step, features and closure
assembly at FP32 accuracy; normalisation, flags and merge bit-exact.
"""
import numpy as np
import pytest

import synth
from oracle import closure as oc

pytestmark = pytest.mark.gpu

NAMES = [n for n, _ in oc.MLP.SHAPES]


def _torch():
    import torch
    return torch


def _t(a, dtype=None):
    torch = _torch()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _bf16_bits(a):
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16).view(np.int16)


def _params(seed, bias_scale=0.1):
    """Random FP32 parameters with He-scaled weights and small biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in oc.MLP.SHAPES:
        if name.startswith("W"):
            fan_in = shp[0]
            d[name] = rng.normal(0, np.sqrt(2.0 / fan_in), shp)
        else:
            d[name] = rng.normal(0, bias_scale, shp)
    flat = np.concatenate([d[n].ravel() for n in NAMES]).astype(np.float32)
    return flat


def _oracle_net(flat32, rnd):
    """The oracle network on the values the GPU sees: BF16 weights, FP32 biases."""
    net = oc.MLP(flat32.astype(np.float64), rnd=rnd)
    for n in NAMES:
        if n.startswith("W"):
            net.p[n] = oc.bf16_round(net.p[n])
    return net


def _relF(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _inputs(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 16)).astype(np.float32)
    X[:, 12:] = 0.0
    return X


@pytest.mark.parametrize("n,use_rows", [(209, False), (1, False), (64, False), (150, True)])
def test_mlp_forward(rt, n, use_rows):
    flat = _params(1)
    net = rt.MLP(seed=0)
    net.set_params(flat)
    X = _inputs(2, 300 if use_rows else n)
    Xb = _bf16_bits(X)
    rows = np.random.default_rng(3).permutation(len(X))[:n].astype(np.int32) if use_rows else None
    Y = net.forward(_t(Xb), rows=None if rows is None else _t(rows)).cpu().numpy().astype(np.float64)
    Xo = oc.bf16_round(X)[rows if use_rows else slice(None)]
    y_m, _ = _oracle_net(flat, oc.bf16_round).forward(Xo)
    y_e, _ = _oracle_net(flat, None).forward(Xo)
    print(f"forward n={n}: rel vs mirrored {_relF(Y, y_m):.2e}, vs unrounded {_relF(Y, y_e):.2e}")
    assert Y.shape == (n, 2)
    assert _relF(Y, y_m) <= 5e-4
    assert _relF(Y, y_e) <= 2e-2
    # inference without stored activations gives the same bits as with them
    Yk = net.forward(_t(Xb), rows=None if rows is None else _t(rows), keep=True).cpu().numpy()
    assert np.array_equal(Yk.astype(np.float64), Y)


@pytest.mark.parametrize("use_rows", [False, True])
def test_mlp_forward_many_samples(rt, use_rows):
    """Above 65 536 samples the forward runs persistent workgroups that keep the hidden
    weights in registers (16x16x32 matrix-core products): the same bars against the oracle,
    a ragged last tile, keep=True bit-identical to keep=False, and every stored
    pre-activation the oracle's (same rounding points) up to a few BF16 rounding flips."""
    torch = _torch()
    flat = _params(11)
    net = rt.MLP(seed=0)
    net.set_params(flat)
    n = 70_001
    X = _inputs(12, 80_000 if use_rows else n)
    Xb = _bf16_bits(X)
    rows = np.random.default_rng(13).integers(0, len(X), n).astype(np.int32) if use_rows else None
    Y = net.forward(_t(Xb), rows=None if rows is None else _t(rows)).cpu().numpy().astype(np.float64)
    Xo = oc.bf16_round(X)[rows if use_rows else slice(None)]
    onet = _oracle_net(flat, oc.bf16_round)
    y_m, _ = onet.forward(Xo)
    y_e, _ = _oracle_net(flat, None).forward(Xo)
    print(f"forward n={n}: rel vs mirrored {_relF(Y, y_m):.2e}, vs unrounded {_relF(Y, y_e):.2e}")
    assert _relF(Y, y_m) <= 5e-4
    assert _relF(Y, y_e) <= 2e-2
    ws = net.workspace(n)
    Yk = net.forward(_t(Xb), rows=None if rows is None else _t(rows), keep=True).cpu().numpy()
    assert np.array_equal(Yk.astype(np.float64), Y)
    # the stored z of the first hidden layer: BF16 values of the oracle's pre-activations
    z1 = ws[: n * 256 * 2].view(torch.int16).cpu().numpy().reshape(n, 256)
    z1 = (z1.astype(np.int32).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    W1 = oc.bf16_round(flat[:16 * 256].astype(np.float64).reshape(16, 256))
    z_ref = oc.bf16_round(Xo @ W1 + flat[16 * 256:16 * 256 + 256].astype(np.float64))
    assert np.mean(z1 != z_ref) < 1e-3


def test_mlp_params_roundtrip(rt):
    flat = _params(4)
    net = rt.MLP(seed=0)
    assert net.n_params() == oc.MLP.n_params() == rt.binding.MLP_NPARAM
    net.set_params(flat)
    assert np.array_equal(net.get_params(), flat)


@pytest.mark.parametrize("n,use_rows", [(200, False), (130, True), (1, False), (33, True)])
def test_mlp_loss_and_gradients(rt, n, use_rows):
    torch = _torch()
    flat = _params(5)
    net = rt.MLP(seed=0)
    net.set_params(flat)
    X = _inputs(6, 256)
    Xb = _t(_bf16_bits(X))
    rng = np.random.default_rng(7)
    T = rng.normal(0, 0.5, 256).astype(np.float32)
    rows = rng.permutation(256)[:n].astype(np.int32) if use_rows else None
    if not use_rows:
        X, T_used = X[:n], T[:n]
        Xb = Xb[:n].contiguous()
    else:
        T_used = T[rows]
    r_t = None if rows is None else _t(rows)
    Y = net.forward(Xb, rows=r_t, n=n, keep=True)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    dY = rt.mlp_nll(Y, _t(T), rows=r_t, n=n, loss_sum=loss)
    Yh = Y.cpu().numpy().astype(np.float64)
    l_o, dy_o = oc.nll_loss(Yh, T_used.astype(np.float64))
    dYh = dY.cpu().numpy().astype(np.float64)
    assert np.allclose(dYh, dy_o, rtol=1e-5, atol=1e-9)
    assert abs(loss.item() / n - l_o) <= 1e-5 * max(1.0, abs(l_o))
    net.zero_grad()
    net.backward(Xb, dY, rows=r_t, n=n)
    g = net.get_grads()
    Xo = oc.bf16_round(X[rows] if use_rows else X)
    for rnd, tol in ((oc.bf16_round, 1e-3), (None, 1e-2)):
        o = _oracle_net(flat, rnd)
        _, cache = o.forward(Xo)
        go = o.flat(o.backward(cache, dYh))
        ofs = 0
        for name, shp in oc.MLP.SHAPES:
            k = int(np.prod(shp))
            e = _relF(g[ofs:ofs + k].astype(np.float64), go[ofs:ofs + k])
            print(f"grad {name} ({'mirrored' if rnd else 'unrounded'}): rel {e:.2e}")
            assert e <= tol, (name, e)
            ofs += k
    # gradients accumulate until zeroed
    net.backward(Xb, dY, rows=r_t, n=n)
    g2 = net.get_grads()
    assert np.allclose(g2, 2 * g, rtol=1e-6, atol=1e-12)


def _grad_errors(g, flat, Xo, dYh):
    out = {}
    for rnd, key in ((oc.bf16_round, "mirrored"), (None, "unrounded")):
        o = _oracle_net(flat, rnd)
        _, cache = o.forward(Xo)
        go = o.flat(o.backward(cache, dYh))
        ofs = 0
        for name, shp in oc.MLP.SHAPES:
            k = int(np.prod(shp))
            out[(name, key)] = _relF(g[ofs:ofs + k].astype(np.float64), go[ofs:ofs + k])
            ofs += k
    return out


def test_mlp_gradients_training_batch(rt):
    """The training batch (8192 samples drawn with replacement): the signal pass runs 256
    workgroups and the weight pass 8 sample chunks per block; same bars as the small batches."""
    torch = _torch()
    flat = _params(21)
    net = rt.MLP(seed=0)
    net.set_params(flat)
    N, n = 20_000, 8192
    X = _inputs(22, N)
    Xb = _t(_bf16_bits(X))
    rng = np.random.default_rng(23)
    T = rng.normal(0, 0.5, N).astype(np.float32)
    rows = rng.integers(0, N, n).astype(np.int32)
    Y = net.forward(Xb, rows=_t(rows), keep=True)
    dY = rt.mlp_nll(Y, _t(T), rows=_t(rows))
    net.zero_grad()
    net.backward(Xb, dY, rows=_t(rows))
    g = net.get_grads()
    errs = _grad_errors(g, flat, oc.bf16_round(X[rows]), dY.cpu().numpy().astype(np.float64))
    for (name, key), e in errs.items():
        print(f"grad {name} ({key}): rel {e:.2e}")
        assert e <= (1e-3 if key == "mirrored" else 1e-2), (name, key, e)
    # deterministic: the same call gives the same bits
    net.zero_grad()
    net.backward(Xb, dY, rows=_t(rows))
    assert np.array_equal(net.get_grads(), g)
    torch.cuda.synchronize()


def test_mlp_gradients_many_samples(rt):
    """70 001 samples: more tiles than signal-pass workgroups (each takes several), 64 sample
    chunks in the weight pass and a ragged last tile; same bars against the oracle."""
    flat = _params(24)
    net = rt.MLP(seed=0)
    net.set_params(flat)
    n = 70_001
    X = _inputs(25, n)
    Xb = _t(_bf16_bits(X))
    T = np.random.default_rng(26).normal(0, 0.5, n).astype(np.float32)
    Y = net.forward(Xb, keep=True)
    dY = rt.mlp_nll(Y, _t(T))
    net.zero_grad()
    net.backward(Xb, dY)
    g = net.get_grads()
    errs = _grad_errors(g, flat, oc.bf16_round(X), dY.cpu().numpy().astype(np.float64))
    for (name, key), e in errs.items():
        print(f"grad {name} ({key}): rel {e:.2e}")
        assert e <= (1e-3 if key == "mirrored" else 1e-2), (name, key, e)


def _splitmix_rows(seed, step, batch, N):
    """Rows of training step `step` by the SplitMix64 finaliser (Steele, Lea and Flood 2014)."""
    M = np.uint64(0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        i = np.arange(batch, dtype=np.uint64)
        z = np.uint64(seed) + (np.uint64(step) * np.uint64(batch) + i + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = (z ^ (z >> np.uint64(31))) & M
    return (z % np.uint64(N)).astype(np.int32)


def test_mlp_train_graph_matches_steps(rt):
    """rt_mlp_train (one captured step, replayed) against the same steps called one at a time
    with the rows drawn by the published SplitMix64 and the cosine learning rate computed on
    the host; split calls continue the step counter.  The schedule is formed in FP64 from the
    FP32 values of lr and lr_final (as the options struct holds them) and rounded to FP32, so
    the host's rates are the device's and all seven steps are bit-identical."""
    import math
    torch = _torch()
    N, batch, total = 3000, 700, 10
    X = _inputs(31, N)
    Xb = _t(_bf16_bits(X))
    T = _t(np.random.default_rng(32).normal(0, 0.5, N).astype(np.float32))
    kw = dict(batch=batch, total_steps=total, lr=2e-3, lr_final=1e-4, wd=1e-3, seed=77)
    one_a, one_b = rt.MLP(seed=5), rt.MLP(seed=5)
    one_a.train(Xb, T, 1, **kw)
    rows0 = _t(_splitmix_rows(77, 0, batch, N))
    Y0 = one_b.forward(Xb, rows=rows0, keep=True)
    one_b.zero_grad()
    one_b.backward(Xb, rt.mlp_nll(Y0, T, rows=rows0), rows=rows0)
    one_b.adam_step(lr=2e-3, wd=1e-3)
    assert np.array_equal(one_a.get_params(), one_b.get_params())
    assert np.array_equal(one_a.get_grads(), one_b.get_grads())
    a = rt.MLP(seed=5)
    la = torch.zeros(1, dtype=torch.float32, device="cuda")
    a.train(Xb, T, 3, loss_sum=la, **kw)
    a.train(Xb, T, 4, loss_sum=la, **kw)
    b = rt.MLP(seed=5)
    lb = torch.zeros(1, dtype=torch.float32, device="cuda")
    lr0, lr1 = float(np.float32(2e-3)), float(np.float32(1e-4))
    for k in range(7):
        rows = _t(_splitmix_rows(77, k, batch, N))
        lr = float(np.float32(lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * (min(k, total) / total)))))
        Y = b.forward(Xb, rows=rows, keep=True)
        dY = rt.mlp_nll(Y, T, rows=rows, loss_sum=lb)
        b.zero_grad()
        b.backward(Xb, dY, rows=rows)
        b.adam_step(lr=lr, wd=1e-3)
    pa, pb = a.get_params(), b.get_params()
    d = float(np.max(np.abs(pa - pb)))
    print(f"graph vs steps: max |dw| {d:.3e}, loss {la.item():.6f} vs {lb.item():.6f}")
    assert np.array_equal(pa, pb)
    # the loss sums are accumulated by atomics (order not fixed)
    assert abs(la.item() - lb.item()) <= 1e-5 * abs(lb.item())
    # one call of 7 steps is the same as 3 + 4
    c = rt.MLP(seed=5)
    c.train(Xb, T, 7, **kw)
    assert np.array_equal(c.get_params(), pa)


def test_adam_steps(rt):
    flat = _params(8)
    net = rt.MLP(seed=0)
    net.set_params(flat)
    X = _inputs(9, 100)
    Xb = _t(_bf16_bits(X))
    T = _t(np.random.default_rng(10).normal(0, 0.5, 100).astype(np.float32))
    Y = net.forward(Xb, keep=True)
    dY = rt.mlp_nll(Y, T)
    net.zero_grad()
    net.backward(Xb, dY)
    g = net.get_grads().astype(np.float64)
    w = flat.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for step in (1, 2):
        net.adam_step(lr=1e-3, wd=1e-2)
        w, m, v = oc.adam_step(w, g, m, v, step, lr=1e-3, wd=1e-2)
        got = net.get_params().astype(np.float64)
        assert np.allclose(got, w, rtol=2e-6, atol=1e-8), float(np.max(np.abs(got - w)))


def test_training_reduces_error(rt):
    """A few hundred Adam steps on a smooth synthetic regression cut the error of m."""
    torch = _torch()
    rng = np.random.default_rng(11)
    n = 8192
    X = _inputs(12, n)
    T = (0.3 * np.sin(2 * X[:, 0]) + 0.1 * X[:, 1] ** 2 - 0.2 * X[:, 2] * X[:, 3]).astype(np.float32)
    Xb = _t(_bf16_bits(X))
    Tt = _t(T)
    net = rt.MLP(seed=3)

    def mse():
        Y = net.forward(Xb).cpu().numpy()
        return float(np.mean((Y[:, 0] - T) ** 2))

    e0 = mse()
    batch = 512
    for step in range(400):
        rows = _t(rng.choice(n, batch, replace=False).astype(np.int32))
        Y = net.forward(Xb, rows=rows, keep=True)
        dY = rt.mlp_nll(Y, Tt, rows=rows)
        net.zero_grad()
        net.backward(Xb, dY, rows=rows)
        net.adam_step(lr=1e-3)
    torch.cuda.synchronize()
    e1 = mse()
    print(f"training: mse {e0:.4f} -> {e1:.5f} (target variance {T.var():.4f})")
    assert e1 < 0.1 * T.var() and e1 < 0.2 * e0


@pytest.mark.parametrize("subset,with_u", [(False, False), (True, False), (False, True), (True, True)])
def test_features(rt, orc, subset, with_u):
    m = synth.tiny_model(21, P=200, F=8)
    chi32, eta32 = m.chi.astype(np.float32), m.eta.astype(np.float32)
    m.chi, m.eta = chi32.astype(np.float64), eta32.astype(np.float64)
    rng = np.random.default_rng(13)
    J1 = rng.uniform(0.05, 2.0, (m.P, m.F)).astype(np.float32)
    u = rng.uniform(0.05, 2.0, (m.P, 6, m.F)).astype(np.float32) if with_u else None
    x = m.freq.x().astype(np.float32)
    e = oc.features(m, J1.astype(np.float64), x.astype(np.float64),
                    None if u is None else u.astype(np.float64)).reshape(m.P, m.F, 16)
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    if subset:
        pts = rng.permutation(m.P)[:77].astype(np.int32)
        got = rt.closure_features(model, _t(chi32), _t(eta32), _t(x), _t(J1[pts]),
                                  u=None if u is None else _t(u[pts]), points=_t(pts))
        e = e[pts]
    else:
        got = rt.closure_features(model, _t(chi32), _t(eta32), _t(x), _t(J1), u=None if u is None else _t(u))
    got = got.cpu().numpy().reshape(e.shape)
    assert np.allclose(got, e, rtol=1e-5, atol=5e-5), float(np.max(np.abs(got - e)))
    rt.sync_status()


def test_features_rejects_bad_point_id(rt):
    m = synth.tiny_model(22, P=50, F=4)
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    J1 = _t(np.ones((2, m.F), np.float32))
    pts = _t(np.array([3, m.P + 5], np.int32))
    x = _t(m.freq.x().astype(np.float32))
    feat = rt.closure_features(model, _t(m.chi.astype(np.float32)), _t(m.eta.astype(np.float32)), x, J1, points=pts)
    with pytest.raises(rt.RtError) as ei:
        rt.sync_status()
    assert ei.value.code == -1
    f = feat.cpu().numpy()
    assert np.all(f[m.F:] == 0) and np.all(np.isfinite(f[:m.F]))


def test_feature_stats_and_normalize(rt):
    rng = np.random.default_rng(14)
    feat = (rng.normal(size=(3001, 16)) * rng.uniform(0.1, 5, 16) + rng.normal(size=16)).astype(np.float32)
    s = rt.closure_feature_stats(_t(feat)).cpu().numpy()
    f64 = feat.astype(np.float64)
    assert np.allclose(s[:16], f64.sum(0), rtol=1e-12, atol=1e-9)
    assert np.allclose(s[16:], (f64 * f64).sum(0), rtol=1e-12, atol=1e-9)
    mean = (s[:16] / len(feat)).astype(np.float32)
    istd = (1.0 / np.sqrt(s[16:] / len(feat) - (s[:16] / len(feat)) ** 2)).astype(np.float32)
    X = rt.closure_normalize(_t(feat), mean, istd).cpu().numpy()
    want = _bf16_bits((feat - mean) * istd)  # FP32 arithmetic, then round to BF16
    assert np.array_equal(X, want)


def test_closure_apply_merge_targets(rt):
    torch = _torch()
    rng = np.random.default_rng(15)
    P, F = 300, 7
    J1 = rng.uniform(0.1, 1.0, (P, F)).astype(np.float32)
    Y = np.stack([rng.normal(0, 0.1, P * F), rng.normal(-6, 1.5, P * F)], 1).astype(np.float32)
    for bound in (np.inf, -np.inf, -3.0, -4.5):
        J, fl, nf = rt.closure_apply(_t(J1), _t(Y), bound)
        Jo, flo = oc.closure_apply(J1.astype(np.float64), Y.astype(np.float64), F, bound)
        n = int(nf.item())
        got = np.sort(fl[:n].cpu().numpy())
        assert np.array_equal(got, np.nonzero(flo)[0])
        assert np.allclose(J.cpu().numpy(), Jo, rtol=2e-6)
        if 0 < n:
            Jf = rng.uniform(5, 6, (n, F)).astype(np.float32)
            rt.closure_merge(_t(Jf), fl, n, J)
            Jh = J.cpu().numpy()
            order = fl[:n].cpu().numpy()
            assert np.array_equal(Jh[order], Jf)
            keep = np.setdiff1d(np.arange(P), order)
            assert np.allclose(Jh[keep], Jo[keep], rtol=2e-6)
    J8 = rng.uniform(0.1, 1.0, (P, F)).astype(np.float32)
    T = rt.closure_targets(_t(J1), _t(J8)).cpu().numpy()
    assert np.allclose(T, np.log(J8.astype(np.float64) / J1).ravel(), rtol=1e-5, atol=1e-6)
    torch.cuda.synchronize()
