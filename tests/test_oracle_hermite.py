"""Pins of the oracle's fourth-order Hermitian Feautrier rows with third-order
boundary conditions (the solver variant Section 2.1 names; rows derived in
oracle.c).  The rows are fixed by what the mathematics forces: exactness for
S = I, the convergence orders on problems with closed forms (fourth order in the
interior, third order with the boundaries), and agreement with an exact
rational elimination of the same tridiagonal system."""
from fractions import Fraction

import numpy as np
import pytest


def _grid(T, n, stretched):
    x = np.linspace(0.0, 1.0, n)
    return T * (x - 0.15 * np.sin(2 * np.pi * x) / (2 * np.pi)) if stretched else T * x


def test_single_point_line(orc):
    assert orc.feautrier_u_hermite([], [0.7], 0, 0.25) == 0.25


def test_steps_beyond_the_limit_give_no_value(orc):
    # uniform steps: the off-diagonal 2/h^2 - 1/12 changes sign at h = 2 sqrt 3
    S = np.full(12, 1.0)
    assert np.isfinite(orc.feautrier_u_hermite(np.full(11, 3.4), S, 5, 0.0))
    assert np.isnan(orc.feautrier_u_hermite(np.full(11, 3.5), S, 5, 0.0))


@pytest.mark.parametrize("dt", [1e-6, 1e-3, 0.3, 2.0])
def test_uniform_source_equal_to_boundary(orc, dt):
    rng = np.random.default_rng(2)
    N = 31
    dtau = dt * rng.uniform(0.7, 1.4, N - 1)
    for m in (0, 7, N - 1):
        assert abs(orc.feautrier_u_hermite(dtau, np.full(N, 0.8125), m, 0.8125) - 0.8125) <= 1e-12


@pytest.mark.parametrize("stretched", [False, True])
def test_interior_fourth_order(orc, stretched):
    # deep inside a slab 60 optical depths thick the boundaries contribute < e^-29: the
    # solution of u'' = u - S with S = 1 + sin(tau/3)/2 is 1 + (9/20) sin(tau/3)
    T, errs = 60.0, []
    for n in (61, 121, 241, 481):
        tau = _grid(T, n, stretched)
        S = 1.0 + 0.5 * np.sin(tau / 3.0)
        m = int(np.argmin(np.abs(tau - T / 2)))
        exact = 1.0 + 0.45 * np.sin(tau[m] / 3.0)
        errs.append(abs(orc.feautrier_u_hermite(np.diff(tau), S, m, 1.0) - exact))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(14.5 < r < 17.5 for r in ratios), ratios


@pytest.mark.parametrize("stretched", [False, True])
def test_third_order_with_boundaries(orc, stretched):
    # slab [0, T], S = s0 + s1 tau, incident I at both ends: u = S + A e^-tau + B e^(tau-T)
    # with A = (I + s1 - s0)/2, B = (I - s0 - s1 (T + 1))/2; the slope of S exercises the
    # third-order term of the boundary rows
    T, s0, s1, I = 5.0, 1.0, 0.4, 0.3
    A, B = (I + s1 - s0) / 2, (I - s0 - s1 * (T + 1)) / 2
    errs, errs2 = [], []
    for n in (21, 41, 81, 161, 321):
        tau = _grid(T, n, stretched)
        S = s0 + s1 * tau
        exact = lambda t: s0 + s1 * t + A * np.exp(-t) + B * np.exp(t - T)
        err = max(abs(orc.feautrier_u_hermite(np.diff(tau), S, m, I) - exact(tau[m])) for m in (0, n // 4, n - 1))
        errs.append(err)
        errs2.append(abs(orc.feautrier_u(np.diff(tau), S, n // 4, I) - exact(tau[n // 4])))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(7.0 < r < 9.0 for r in ratios), ratios
    assert errs[-1] < errs2[-1] / 4  # below the second-order scheme on the same grid


def _rows_exact(dtau, S, I):
    """The Hermitian system in exact rationals (same rows as the oracle's comment)."""
    F = Fraction
    N = len(S)
    d = [F(float(x)) for x in dtau]
    s = [F(float(x)) for x in S]
    Ii = F(float(I))
    M = [[F(0)] * N for _ in range(N)]
    r = [F(0)] * N
    for k in range(N):
        if k in (0, N - 1):
            dt = d[0] if k == 0 else d[N - 2]
            nb = 1 if k == 0 else N - 2
            E = (2 / dt) * (1 + dt * dt / 6)
            K = 2 / (dt * dt)
            M[k][k] = 1 + E + K
            M[k][nb] = -K
            r[k] = s[k] + E * Ii + (s[nb] - s[k]) / 3
        else:
            a, b = d[k - 1], d[k]
            h = (a + b) / 2
            al = (a ** 3 + 2 * a * a * b - b ** 3) / (12 * a * (a + b)) / h
            ga = (b ** 3 + 2 * a * b * b - a ** 3) / (12 * b * (a + b)) / h
            A, C = 2 / (a * (a + b)), 2 / (b * (a + b))
            M[k][k - 1] = -(A - al)
            M[k][k + 1] = -(C - ga)
            M[k][k] = 1 + (A - al) + (C - ga)
            r[k] = al * s[k - 1] + (1 - al - ga) * s[k] + ga * s[k + 1]
    return M, r


def _solve_exact(M, r):
    N = len(r)
    M = [row[:] for row in M]
    r = r[:]
    for c in range(N):
        p = next(i for i in range(c, N) if M[i][c] != 0)
        M[c], M[p] = M[p], M[c]
        r[c], r[p] = r[p], r[c]
        for i in range(c + 1, N):
            q = M[i][c] / M[c][c]
            if q:
                for j in range(c, N):
                    M[i][j] -= q * M[c][j]
                r[i] -= q * r[c]
    x = [Fraction(0)] * N
    for i in reversed(range(N)):
        x[i] = (r[i] - sum(M[i][j] * x[j] for j in range(i + 1, N))) / M[i][i]
    return x


@pytest.mark.parametrize("seed", range(6))
def test_elimination_matches_exact_rational_solve(orc, seed):
    # the elimination, not the rows: the rescaled two-sided sweep against exact Gaussian
    # elimination, for steps below the sign-change limit
    rng = np.random.default_rng(40 + seed)
    N = int(rng.integers(2, 14))
    dtau = 10.0 ** rng.uniform(-3, 0.4, N - 1)
    S = rng.uniform(0.1, 2.0, N)
    I = float(rng.uniform(0, 1))
    x = _solve_exact(*_rows_exact(dtau, S, I))
    for m in sorted({0, N - 1, int(rng.integers(0, N))}):
        u = orc.feautrier_u_hermite(dtau, S, m, I)
        assert abs(Fraction(u) - x[m]) <= Fraction(1, 10 ** 11) * abs(x[m]), (N, m, u, float(x[m]))


def test_full_path_uniform_source(orc):
    """Through line assembly, Doppler shifts and both sides: S uniform and equal to
    the incident intensity gives J = S with the Hermitian rows too."""
    import synth
    m = synth.tiny_model(9, P=50, F=12, moving=True)
    S0 = 0.625
    m.eta = m.chi * S0
    m.I_bc = np.full(m.F, S0)
    _, dirs, w2 = orc.dirset_uniform(2)
    J = orc.compute_J(m, dirs, w2, scheme=1, dtau_max=0.5)  # steps within the rows' limit
    assert np.max(np.abs(J - S0)) < 1e-12
    with pytest.raises(FloatingPointError):  # this model's whole steps exceed it
        orc.compute_J(m, dirs, w2, scheme=1)


def test_full_path_switch_reaches_the_solve(orc):
    """On the homogeneous sphere with a source varying smoothly in space (optical-depth
    steps ~0.2) the two schemes differ by their truncation error: more than rounding,
    less than a few per cent."""
    import synth
    m = synth.sphere_model(F=3)
    r = np.linalg.norm(m.pos, axis=1)
    m.eta = m.chi * (1.0 + 0.5 * np.cos(2.0 * r))[:, None]
    _, dirs, w2 = orc.dirset_uniform(1)
    org = np.arange(0, m.P, 97, dtype=np.int32)
    J2 = orc.compute_J(m, dirs, w2, origins=org)
    J4 = orc.compute_J(m, dirs, w2, origins=org, scheme=1)
    d = np.max(np.abs(J4 - J2) / np.abs(J2))
    assert 1e-8 < d < 0.05, d
