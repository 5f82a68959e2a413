"""FP64 reference of the learned closure: features, MLP forward/backward, loss,
Adam step and the fallback rule.

TEST INFRASTRUCTURE ONLY (used by tests and the benchmark's CPU leg).  Plain
numpy; no code shared with the HIP library.

Closure (the build's addition to the method): a cheap J at nside = 1 plus local
optical properties are mapped by a small MLP to the J of the fine direction set
(nside = 8).  Per (point p, frequency f) sample:

features (in this order; computed from the model, J1 = J at nside 1):
   0  log J1[p,f]
   1  log chi[p,f]
   2  log S[p,f],  S = eta/chi
   3  mean over neighbours n of log chi[n,f]
   4  mean over neighbours of log S[n,f]
   5  standard deviation over neighbours of log chi[n,f]
   6  Gf_p(chi) = max_n |(chi_p - chi_n)/(chi_p + chi_n)|    (eq. 6)
   7  Gf_p(S)                                                (eq. 6)
   8  log L_p, L_p = mean_n |x_p - x_n|                      (eq. 8)
   9  log(chi[p,f] L_p)
  10  x_f / 5                (frequency in Doppler widths)
  11  log(number of neighbours)
  12  max over the R coarse pairs r of log(u_r[p,f] / J1[p,f])   (u: per-pair mean
  13  min over r of the same                                    intensities of the
  14  standard deviation over r of the same                    coarse solve; zero
                                                                when not given)
  15  zero (padding to 16)

network: h1 = silu(x W1 + b1), h2 = silu(h1 W2 + b2), h3 = silu(h2 W3 + b3),
         y = h3 W4 + b4, y = (m, s): m predicts log(J8/J1), s the log variance of
         its error.  silu(z) = z / (1 + exp(-z)).
loss (per sample): 0.5 (exp(-s) (t - m)^2 + s),  t = log(J8/J1); mean over samples.
closure: J = J1 exp(m); a point falls back to the plain fine solve when for some
         frequency 0.5 s > log(bound) (predicted |log error| above the bound).
"""
from __future__ import annotations

import numpy as np

D_IN = 16
N_FEAT = 12


def features(model, J1: np.ndarray, freq_x: np.ndarray, u: np.ndarray = None) -> np.ndarray:
    """[P*F][16] features, sample index p*F + f; u optional [P][R][F]."""
    P, F = model.P, J1.shape[1]
    chi = np.asarray(model.chi, np.float64)
    S = np.asarray(model.eta, np.float64) / chi
    off, idx, pos = model.nbr_off, model.nbr_idx, model.pos
    X = np.zeros((P, F, D_IN))
    lchi, lS = np.log(chi), np.log(S)
    for p in range(P):
        nb = idx[off[p]:off[p + 1]]
        L = np.mean(np.linalg.norm(pos[nb] - pos[p], axis=1))
        X[p, :, 0] = np.log(J1[p])
        X[p, :, 1] = lchi[p]
        X[p, :, 2] = lS[p]
        X[p, :, 3] = lchi[nb].mean(0)
        X[p, :, 4] = lS[nb].mean(0)
        X[p, :, 5] = lchi[nb].std(0)
        X[p, :, 6] = np.max(np.abs((chi[p] - chi[nb]) / (chi[p] + chi[nb])), 0)
        X[p, :, 7] = np.max(np.abs((S[p] - S[nb]) / (S[p] + S[nb])), 0)
        X[p, :, 8] = np.log(L)
        X[p, :, 9] = np.log(chi[p] * L)
        X[p, :, 10] = np.asarray(freq_x) / 5.0
        X[p, :, 11] = np.log(len(nb))
        if u is not None:
            a = np.log(u[p]) - np.log(J1[p])[None, :]   # [R][F]
            X[p, :, 12] = a.max(0)
            X[p, :, 13] = a.min(0)
            X[p, :, 14] = a.std(0)
    return X.reshape(P * F, D_IN)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


class MLP:
    """Parameters as a dict of float64 arrays: W1 [16,256], b1, W2, b2, W3, b3, W4 [256,2], b4.

    rnd (optional) is applied where a reduced-precision implementation stores a
    value: the pre-activations z, the activations silu(z) and the backward
    signals dz (pass bf16_round to mirror a BF16 matrix-core implementation; the
    weights and inputs are rounded by the caller).  The default stores exactly.
    """

    SHAPES = (("W1", (D_IN, 256)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
              ("W3", (256, 256)), ("b3", (256,)), ("W4", (256, 2)), ("b4", (2,)))

    def __init__(self, flat: np.ndarray, rnd=None):
        self.rnd = rnd if rnd is not None else (lambda a: a)
        self.p = {}
        o = 0
        for name, shp in self.SHAPES:
            n = int(np.prod(shp))
            self.p[name] = np.asarray(flat[o:o + n], np.float64).reshape(shp)
            o += n
        assert o == len(flat)

    @classmethod
    def n_params(cls) -> int:
        return sum(int(np.prod(s)) for _, s in cls.SHAPES)

    def flat(self, d=None) -> np.ndarray:
        d = self.p if d is None else d
        return np.concatenate([d[n].ravel() for n, _ in self.SHAPES])

    def forward(self, X):
        p, r = self.p, self.rnd
        z1 = r(X @ p["W1"] + p["b1"])
        h1 = r(silu(z1))
        z2 = r(h1 @ p["W2"] + p["b2"])
        h2 = r(silu(z2))
        z3 = r(h2 @ p["W3"] + p["b3"])
        h3 = r(silu(z3))
        y = h3 @ p["W4"] + p["b4"]
        return y, (X, z1, h1, z2, h2, z3, h3)

    def backward(self, cache, dy):
        """Gradients of sum(dy * y) with respect to every parameter."""
        X, z1, h1, z2, h2, z3, h3 = cache
        p, r = self.p, self.rnd
        g = {}
        g["W4"] = h3.T @ dy
        g["b4"] = dy.sum(0)
        dz3 = r((dy @ p["W4"].T) * dsilu(z3))
        g["W3"] = h2.T @ dz3
        g["b3"] = dz3.sum(0)
        dz2 = r((dz3 @ p["W3"].T) * dsilu(z2))
        g["W2"] = h1.T @ dz2
        g["b2"] = dz2.sum(0)
        dz1 = r((dz2 @ p["W2"].T) * dsilu(z1))
        g["W1"] = X.T @ dz1
        g["b1"] = dz1.sum(0)
        return g


def nll_loss(y, t):
    """Mean Gaussian negative log-likelihood and its gradient with respect to y."""
    m, s = y[:, 0], y[:, 1]
    e = np.exp(-s)
    r = t - m
    loss = 0.5 * (e * r * r + s)
    n = len(t)
    dy = np.stack([-(e * r) / n, 0.5 * (1.0 - e * r * r) / n], 1)
    return loss.mean(), dy


def adam_step(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One Adam update (with decoupled weight decay); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v


def closure_apply(J1, y, F, log_bound):
    """J = J1 exp(m) per (point, f); flagged[p] when any 0.5 s > log_bound."""
    m = y[:, 0].reshape(-1, F)
    s = y[:, 1].reshape(-1, F)
    J = J1 * np.exp(m)
    flagged = np.any(0.5 * s > log_bound, axis=1)
    return J, flagged


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
