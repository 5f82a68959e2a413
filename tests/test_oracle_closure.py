"""Pins of the closure oracle: gradients by central finite differences, the loss
and its gradient in closed form, features against direct definitions, the
fallback rule's limits."""
import numpy as np
import pytest

import synth
from oracle import closure as oc


def _mlp(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return oc.MLP(rng.normal(0, scale, oc.MLP.n_params()) / np.sqrt(16))


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    assert np.allclose(oc.dsilu(z), (oc.silu(z + h) - oc.silu(z - h)) / (2 * h), atol=1e-8)
    assert oc.silu(0.0) == 0.0 and abs(oc.silu(50.0) - 50.0) < 1e-12


def test_backward_matches_finite_differences():
    net = _mlp(1)
    rng = np.random.default_rng(2)
    X = rng.normal(size=(7, 16))
    dy = rng.normal(size=(7, 2))
    y, cache = net.forward(X)
    g = net.backward(cache, dy)
    flat = net.flat()
    gflat = net.flat(g)
    idx = rng.choice(len(flat), 60, replace=False)
    for i in idx:
        h = 1e-6
        fp = flat.copy()
        fp[i] += h
        fm = flat.copy()
        fm[i] -= h
        yp, _ = oc.MLP(fp).forward(X)
        ym, _ = oc.MLP(fm).forward(X)
        fd = ((yp - ym) * dy).sum() / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gflat[i])


def test_nll_loss_gradient():
    rng = np.random.default_rng(3)
    y = rng.normal(size=(9, 2))
    t = rng.normal(size=9)
    loss, dy = oc.nll_loss(y, t)
    # closed form at one sample: 0.5 (e^-s (t-m)^2 + s)
    m, s = y[0]
    assert np.isclose(0.5 * (np.exp(-s) * (t[0] - m) ** 2 + s), 0.5 * (np.exp(-y[:, 1]) * (t - y[:, 0]) ** 2 + y[:, 1])[0])
    for i in range(9):
        for j in range(2):
            h = 1e-6
            yp, ym = y.copy(), y.copy()
            yp[i, j] += h
            ym[i, j] -= h
            fd = (oc.nll_loss(yp, t)[0] - oc.nll_loss(ym, t)[0]) / (2 * h)
            assert abs(fd - dy[i, j]) < 1e-8
    # at the optimum for fixed m the log-variance equals log of the squared error
    r = 0.37
    s_opt = np.log(r * r)
    _, d = oc.nll_loss(np.array([[0.0, s_opt]]), np.array([r]))
    assert abs(d[0, 1]) < 1e-12


def test_adam_first_step_is_signed_lr():
    w = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    w1, m, v = oc.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(w1, w - 0.01 * np.sign(g))


def test_features_definitions():
    m = synth.tiny_model(20, P=30, F=5)
    rng = np.random.default_rng(4)
    J1 = rng.uniform(0.1, 1.0, (m.P, m.F))
    x = m.freq.x()
    X = oc.features(m, J1, x).reshape(m.P, m.F, 16)
    p, f = 7, 3
    nb = m.nbr_idx[m.nbr_off[p]:m.nbr_off[p + 1]]
    S = m.eta / m.chi
    assert np.isclose(X[p, f, 0], np.log(J1[p, f]))
    assert np.isclose(X[p, f, 6], max(abs((m.chi[p, f] - m.chi[n, f]) / (m.chi[p, f] + m.chi[n, f])) for n in nb))
    assert 0 <= X[:, :, 6].min() and X[:, :, 6].max() <= 1 and X[:, :, 7].max() <= 1  # eq. 6: Gf in [0, 1]
    L = np.mean([np.linalg.norm(m.pos[p] - m.pos[n]) for n in nb])
    assert np.isclose(X[p, f, 8], np.log(L))                                          # eq. 8
    assert np.isclose(X[p, f, 5], np.std([np.log(m.chi[n, f]) for n in nb]))
    assert np.isclose(X[p, f, 4], np.mean([np.log(S[n, f]) for n in nb]))
    assert np.isclose(X[p, f, 10], x[f] / 5) and np.all(X[:, :, 12:] == 0)
    # coarse per-pair intensities: an isotropic field has no spread; one bright pair of six
    u = np.repeat(J1[:, None, :], 6, axis=1)
    Xi = oc.features(m, J1, x, u).reshape(m.P, m.F, 16)
    assert np.allclose(Xi[:, :, 12:15], 0.0, atol=1e-15)
    u[p, 2, f] = 7.0 * J1[p, f]
    Xa = oc.features(m, J1, x, u).reshape(m.P, m.F, 16)
    assert np.isclose(Xa[p, f, 12], np.log(7.0)) and np.isclose(Xa[p, f, 13], 0.0)
    assert np.isclose(Xa[p, f, 14], np.log(7.0) * np.sqrt(5.0) / 6.0)   # one of six at log 7
    # a uniform medium has no gradients
    m.chi[:] = 2.0
    m.eta[:] = 3.0
    Xu = oc.features(m, J1, x).reshape(m.P, m.F, 16)
    assert np.all(Xu[:, :, 6] == 0) and np.all(Xu[:, :, 7] == 0) and np.allclose(Xu[:, :, 5], 0)


def test_closure_apply_limits():
    rng = np.random.default_rng(5)
    J1 = rng.uniform(0.1, 1, (4, 3))
    y = rng.normal(size=(12, 2))
    J, fl = oc.closure_apply(J1, y, 3, np.inf)
    assert not fl.any() and np.allclose(J, J1 * np.exp(y[:, 0].reshape(4, 3)))
    _, fl = oc.closure_apply(J1, y, 3, -np.inf)
    assert fl.all()
    y[:, 0] = 0.0
    J, _ = oc.closure_apply(J1, y, 3, 0.0)
    assert np.array_equal(J, J1)


def test_bf16_rounding():
    a = np.array([1.0, 1.00390625, 1.005859375, -3.14159, 65504.0, 1e-30])
    r = oc.bf16_round(a)
    assert r[0] == 1.0 and r[1] == 1.0  # 1 + 2^-8 ties to even -> 1
    assert r[2] == 1.0078125            # rounds up
    assert abs(r[3] + 3.140625) < 1e-12
    assert np.all(np.abs(r - a) <= np.abs(a) * 2 ** -8)


def test_storage_rounding_hook():
    """With BF16 storage the stored values are representable and the output moves
    by no more than a few BF16 ulps relative; the identity hook changes nothing."""
    net = _mlp(6, scale=1.0)
    rng = np.random.default_rng(7)
    X = rng.normal(size=(33, 16))
    y, _ = net.forward(X)
    r = oc.MLP(net.flat(), rnd=oc.bf16_round)
    yr, cache = r.forward(X)
    for a in cache[1:]:
        assert np.array_equal(oc.bf16_round(a), a)
    assert np.linalg.norm(yr - y) <= 3 * 2.0 ** -8 * np.linalg.norm(y) * 4
    g = r.backward(cache, rng.normal(size=(33, 2)))
    assert all(np.all(np.isfinite(v)) for v in g.values())
    y_id, _ = oc.MLP(net.flat(), rnd=lambda a: a).forward(X)
    assert np.array_equal(y_id, y)
