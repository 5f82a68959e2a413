"""Pins of the oracle's Feautrier solve (eq. 1, second-order boundary
conditions of Section 2.1) against exact rational solves and closed forms."""
from fractions import Fraction

import numpy as np
import pytest
from exact_feautrier import exact_u as _exact_u


@pytest.mark.parametrize("seed", range(12))
def test_rational_solve(orc, seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 24))
    lo = [-7, -4, -2, -1][seed % 4]
    dtau = 10.0 ** rng.uniform(lo, 1.0, N - 1)
    S = rng.uniform(0.0, 2.0, N)
    I = float(rng.uniform(0, 1))
    for m in sorted({0, N - 1, int(rng.integers(0, N))}):
        u = orc.feautrier_u(dtau, S, m, I)
        ue = _exact_u(dtau, S, m, I)
        assert abs(Fraction(u) - ue) <= Fraction(1, 10 ** 13) * abs(ue), (N, m, u, float(ue))


def test_single_point_line(orc):
    assert orc.feautrier_u([], [0.7], 0, 0.25) == 0.25


@pytest.mark.parametrize("dt", [1e-8, 1e-4, 0.3, 5.0, 200.0])
def test_uniform_source_equal_to_boundary(orc, dt):
    # u = S everywhere solves the discrete system exactly when S = I.
    rng = np.random.default_rng(1)
    N = 37
    dtau = dt * rng.uniform(0.5, 2.0, N - 1)
    S = np.full(N, 0.8125)
    for m in (0, 5, N - 1):
        assert abs(orc.feautrier_u(dtau, S, m, 0.8125) - 0.8125) <= 1e-13


def test_constant_step_closed_form(orc):
    # constant dtau h: interior solution u_d = S + a lam^d + b lam^-d,
    # lam + 1/lam = 2 + h^2; a, b from the two boundary rows.
    h, N, S, I = 0.3, 25, 1.3, 0.4
    lam = ((2 + h * h) - np.sqrt((2 + h * h) ** 2 - 4)) / 2
    d = np.arange(N)

    def row0(a, b, dd, nb):
        v0 = a * lam ** dd + b * lam ** -dd
        v1 = a * lam ** nb + b * lam ** -nb
        return (1 + 2 / h + 2 / h ** 2) * v0 - (2 / h ** 2) * v1

    # boundary rows in v = u - S: row0(v) = 2 (I - S)/h at both ends
    M = np.array([[row0(1, 0, 0, 1), row0(0, 1, 0, 1)],
                  [row0(1, 0, N - 1, N - 2), row0(0, 1, N - 1, N - 2)]])
    a, b = np.linalg.solve(M, [2 * (I - S) / h, 2 * (I - S) / h])
    u_cf = S + a * lam ** d + b * lam ** -d
    for m in (0, 3, 12, N - 1):
        u = orc.feautrier_u(np.full(N - 1, h), np.full(N, S), m, I)
        assert u == pytest.approx(u_cf[m], rel=1e-12)


def test_slab_second_order_convergence(orc):
    # homogeneous slab of depth T, no incident light: u(tau) = S (1 - (e^-tau + e^-(T-tau))/2)
    T, S = 6.0, 1.0
    errs = []
    for n in (21, 41, 81, 161, 321):
        h = T / (n - 1)
        m = n // 4
        tau = m * h
        exact = S * (1 - 0.5 * (np.exp(-tau) + np.exp(-(T - tau))))
        u = orc.feautrier_u(np.full(n - 1, h), np.full(n, S), m, 0.0)
        errs.append(abs(u - exact))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.6 < r < 4.4 for r in ratios), ratios
    assert errs[-1] < 1e-4


def test_linearity(orc):
    rng = np.random.default_rng(4)
    N = 30
    dtau = 10 ** rng.uniform(-3, 0.5, N - 1)
    S1, S2 = rng.uniform(0, 1, N), rng.uniform(0, 1, N)
    for m in (0, 11, N - 1):
        u = orc.feautrier_u(dtau, 2 * S1 + 3 * S2, m, 2 * 0.2 + 3 * 0.7)
        u1 = orc.feautrier_u(dtau, S1, m, 0.2)
        u2 = orc.feautrier_u(dtau, S2, m, 0.7)
        assert u == pytest.approx(2 * u1 + 3 * u2, rel=1e-13)


def test_optically_thick_and_thin_limits(orc):
    N = 21
    S = np.linspace(0.5, 1.5, N)
    # very thick: local source
    u = orc.feautrier_u(np.full(N - 1, 1e4), S, 10, 0.0)
    assert u == pytest.approx(S[10], rel=1e-6)
    # very thin: boundary intensity
    u = orc.feautrier_u(np.full(N - 1, 1e-7), S, 10, 0.3)
    assert u == pytest.approx(0.3, rel=1e-5)
