"""Pins of the oracle's adaptive optical-depth increments (Section 2.1.2, eq. 2):
an interval of the line is split into ceil(max(chi) ds / dtau_max) equal parts
with chi and eta interpolated linearly."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import synth
from exact_feautrier import exact_u, exact_u_tridiag


def test_large_bound_changes_nothing(orc):
    """With dtau_max above every interval's optical depth no interval is split: the
    result is the unrefined one, bit for bit."""
    m = synth.tiny_model(5, P=60, F=6, moving=True)
    _, dirs, w2 = orc.dirset_uniform(1)
    J0 = orc.compute_J(m, dirs, w2)
    J1 = orc.compute_J(m, dirs, w2, dtau_max=1e6)
    assert np.array_equal(J0, J1)
    J2 = orc.compute_J(m, dirs, w2, dtau_max=0.05)
    assert not np.allclose(J0, J2, rtol=1e-6)


def test_uniform_source_equal_to_boundary_still_exact(orc):
    """S = I everywhere: u = S on any refined line too."""
    m = synth.tiny_model(6, P=50, F=5, moving=True)
    S = 0.7
    m.eta = m.chi * S
    m.I_bc = np.full(m.F, S)
    _, dirs, w2 = orc.dirset_uniform(1)
    J = orc.compute_J(m, dirs, w2, dtau_max=0.02)
    assert np.allclose(J, S, rtol=1e-12, atol=0)


def test_slab_converges_at_second_order_in_dtau_max(orc):
    """A homogeneous line sampled coarsely (dtau = 1.5 per interval): the error against
    the slab's closed form falls ~4x per halving of dtau_max, and without sub-steps it
    is far larger."""
    n = 21
    m = synth.lattice_model(n=n, F=1, spacing=0.5)
    chi = 3.0
    m.chi[:] = chi
    m.eta[:] = chi * 1.0
    lin = lambda i, j, k: (i * n + j) * n + k  # noqa: E731
    o = lin(6, 0, 0)
    d = np.array([[1.0, 0.0, 0.0]])
    T = chi * 0.5 * (n - 1)
    tau = chi * 0.5 * 6
    exact = 1 - 0.5 * (np.exp(-tau) + np.exp(-(T - tau)))
    e_whole = abs(orc.compute_J(m, d, np.array([1.0]), origins=[o])[0, 0] - exact)
    errs = []
    for dt in (0.4, 0.2, 0.1, 0.05):
        J = orc.compute_J(m, d, np.array([1.0]), origins=[o], dtau_max=dt)
        errs.append(abs(J[0, 0] - exact))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.3 < r < 4.7 for r in ratios), (ratios, errs)
    assert e_whole > 20 * errs[-1]


def _refined_exact_u(trace_ray, m, o, d, f, I, dtau_max, max_sub=1024):
    """u at origin o for pair direction d and frequency f: both rays traced, the line
    assembled, optics shifted and interpolated in the origin's frame along +d, every
    interval split per eq. 2 and interpolated linearly, trapezoid optical depths, exact
    rational solve.  Returns (u, smallest distance of a split count's argument to an
    integer, largest sub-interval dtau)."""
    ids_p, Z_p = trace_ray(m, o, d)
    ids_m, Z_m = trace_ray(m, o, -d)
    q = list(ids_m[::-1]) + [o] + list(ids_p)
    s = [-Fr(float(z)) for z in Z_m[::-1]] + [Fr(0)] + [Fr(float(z)) for z in Z_p]
    mi = len(ids_m)
    starts = np.concatenate([[0], np.cumsum(m.freq.len)])
    b = int(np.searchsorted(starts, f, side="right") - 1)
    fb, L, dx = int(starts[b]), int(m.freq.len[b]), Fr(float(m.freq.dx[b]))
    j = f - fb
    vo = [Fr(float(v)) for v in m.vel[o]]
    dd = [Fr(float(c)) for c in d]
    chi, eta = [], []
    for p in q:
        dv = [Fr(float(v)) - w for v, w in zip(m.vel[p], vo)]
        delta = sum(a * c for a, c in zip(dd, dv)) / dx
        k = math.floor(delta)
        t = delta - k
        ia = min(max(j - k, 0), L - 1)
        ib = min(max(j - k - 1, 0), L - 1)
        chi.append((1 - t) * Fr(float(m.chi[p, fb + ia])) + t * Fr(float(m.chi[p, fb + ib])))
        eta.append((1 - t) * Fr(float(m.eta[p, fb + ia])) + t * Fr(float(m.eta[p, fb + ib])))
    dtm = Fr(dtau_max)
    rc, re, rs, mref = [], [], [], None
    gap = 1.0
    for i in range(len(q)):
        if i == mi:
            mref = len(rc)
        rc.append(chi[i])
        re.append(eta[i])
        rs.append(s[i])
        if i + 1 == len(q):
            break
        arg = max(chi[i], chi[i + 1]) * (s[i + 1] - s[i]) / dtm
        gap = min(gap, abs(float(arg) - round(float(arg))))
        n = min(max(math.ceil(arg), 1), max_sub)
        for k in range(1, n):
            w = Fr(k, n)
            rc.append((1 - w) * chi[i] + w * chi[i + 1])
            re.append((1 - w) * eta[i] + w * eta[i + 1])
            rs.append(s[i] + w * (s[i + 1] - s[i]))
    dtau = [(rc[i] + rc[i + 1]) / 2 * (rs[i + 1] - rs[i]) for i in range(len(rc) - 1)]
    S = [e / c for e, c in zip(re, rc)]
    return exact_u_tridiag(dtau, S, mref, Fr(float(I))), gap, float(max(dtau))


def test_tridiagonal_checker_matches_dense():
    rng = np.random.default_rng(3)
    for N in (2, 3, 9):
        dt = rng.uniform(0.01, 2.0, N - 1)
        S = rng.uniform(0.1, 1.0, N)
        for mm in (0, N // 2, N - 1):
            assert exact_u(dt, S, mm, 0.3) == exact_u_tridiag(dt, S, mm, 0.3)


@pytest.mark.parametrize("dtau_max", [0.35, 0.15])
def test_refined_line_exact(orc, dtau_max):
    """Moving medium, two frequency blocks: the oracle's per-pair u with sub-steps against
    the exact rational construction, and every sub-interval within dtau_max."""
    m = synth.tiny_model(33, P=40, F=8, moving=True)
    m.freq = synth.FreqGrid(np.array([5, 3], np.int32), np.array([-3.0, -1.0]), np.array([0.8, 0.55]))
    rng = np.random.default_rng(9)
    m.chi = m.chi * 2.0
    m.eta = m.eta * 2.0
    m.I_bc = rng.uniform(0.0, 0.4, m.F)
    _, dirs, w2 = orc.dirset_uniform(1)
    origins = np.array([4, 21], np.int32)
    J, u = orc.compute_J(m, dirs, w2, origins=origins, want_u=True, dtau_max=dtau_max)
    checked = 0
    for oi, o in enumerate(origins):
        for r in (1, 4):
            for f in (0, 5, 7):
                ue, gap, dmax = _refined_exact_u(orc.trace_ray, m, int(o), dirs[r], f, m.I_bc[f], dtau_max)
                assert dmax <= dtau_max * (1 + 1e-12)
                if gap < 1e-9:  # a split count on the edge of an integer: FP64 may round either way
                    continue
                assert abs(u[oi, r, f] - float(ue)) <= 1e-12 * abs(float(ue)), (o, r, f)
                checked += 1
    assert checked >= 10


# ----------------------------------------------------------------------------- velocity sampling (Section 2.1.1)

def _sampled_exact_u(trace_ray, m, o, d, f, I, dv_max, dtau_max=0.0, max_sub=1024):
    """Exact rational construction with velocity sampling: assembled points get their
    projected velocity p; an interval whose |p_{d+1} - p_d| exceeds dv_max gets
    ceil(|dp|/dv_max) equal parts whose points carry the interpolated velocity and the
    weight-mixed optics of the two end points, each read at the new point's own shift;
    then the optical-depth split (if any) and the exact solve.  Returns (u, gap) with gap
    the smallest distance of a split argument to an integer."""
    ids_p, Z_p = trace_ray(m, o, d)
    ids_m, Z_m = trace_ray(m, o, -d)
    q = list(ids_m[::-1]) + [o] + list(ids_p)
    s = [-Fr(float(z)) for z in Z_m[::-1]] + [Fr(0)] + [Fr(float(z)) for z in Z_p]
    mi = len(ids_m)
    starts = np.concatenate([[0], np.cumsum(m.freq.len)])
    b = int(np.searchsorted(starts, f, side="right") - 1)
    fb, L, dx = int(starts[b]), int(m.freq.len[b]), Fr(float(m.freq.dx[b]))
    j = f - fb
    vo = [Fr(float(v)) for v in m.vel[o]]
    dd = [Fr(float(c)) for c in d]
    pv = [sum(a * (Fr(float(v)) - w) for a, v, w in zip(dd, m.vel[p], vo)) for p in q]

    def table(p, tab, shift):
        k = math.floor(shift)
        t = shift - k
        ia = min(max(j - k, 0), L - 1)
        ib = min(max(j - k - 1, 0), L - 1)
        return (1 - t) * Fr(float(tab[p, fb + ia])) + t * Fr(float(tab[p, fb + ib]))

    gap = 1.0
    chi, eta, ds, mref = [], [], [], None
    for i in range(len(q)):
        if i == mi:
            mref = len(chi)
        sh = pv[i] / dx
        chi.append(table(q[i], m.chi, sh))
        eta.append(table(q[i], m.eta, sh))
        if i + 1 == len(q):
            break
        arg = abs(pv[i + 1] - pv[i]) / Fr(dv_max)
        gap = min(gap, abs(float(arg) - round(float(arg))))
        n = min(max(math.ceil(arg), 1), max_sub)
        h = (s[i + 1] - s[i]) / n
        ds.append(h)
        for k in range(1, n):
            w = Fr(k, n)
            sh = ((1 - w) * pv[i] + w * pv[i + 1]) / dx
            chi.append((1 - w) * table(q[i], m.chi, sh) + w * table(q[i + 1], m.chi, sh))
            eta.append((1 - w) * table(q[i], m.eta, sh) + w * table(q[i + 1], m.eta, sh))
            ds.append(h)
    rc, re, rds, mr = [], [], [], None
    for i in range(len(chi)):
        if i == mref:
            mr = len(rc)
        rc.append(chi[i])
        re.append(eta[i])
        if i + 1 == len(chi):
            break
        n = 1
        if dtau_max > 0:
            arg = max(chi[i], chi[i + 1]) * ds[i] / Fr(dtau_max)
            gap = min(gap, abs(float(arg) - round(float(arg))))
            n = min(max(math.ceil(arg), 1), max_sub)
        for k in range(1, n):
            w = Fr(k, n)
            rc.append((1 - w) * chi[i] + w * chi[i + 1])
            re.append((1 - w) * eta[i] + w * eta[i + 1])
        rds += [ds[i] / n] * n
    dtau = [(rc[i] + rc[i + 1]) / 2 * rds[i] for i in range(len(rc) - 1)]
    S = [e / c for e, c in zip(re, rc)]
    return exact_u_tridiag(dtau, S, mr, Fr(float(I))), gap


def test_velocity_sampling_identities(orc):
    m = synth.tiny_model(51, P=60, F=6, moving=True)
    _, dirs, w2 = orc.dirset_uniform(1)
    J0 = orc.compute_J(m, dirs, w2)
    assert np.array_equal(J0, orc.compute_J(m, dirs, w2, dv_max=1e6))      # nothing to split
    assert not np.allclose(J0, orc.compute_J(m, dirs, w2, dv_max=0.2), rtol=1e-6)
    ms = synth.tiny_model(51, P=60, F=6, moving=False)                      # static: no velocities to sample
    assert np.array_equal(orc.compute_J(ms, dirs, w2), orc.compute_J(ms, dirs, w2, dv_max=0.1))
    S = 0.4                                                                  # S = I: still exactly S
    m.eta = m.chi * S
    m.I_bc = np.full(m.F, S)
    assert np.allclose(orc.compute_J(m, dirs, w2, dv_max=0.1, dtau_max=0.05), S, rtol=1e-12, atol=0)


@pytest.mark.parametrize("dv_max,dtau_max", [(0.5, 0.0), (0.25, 0.4)])
def test_velocity_sampled_line_exact(orc, dv_max, dtau_max):
    m = synth.tiny_model(52, P=40, F=8, moving=True)
    m.freq = synth.FreqGrid(np.array([5, 3], np.int32), np.array([-3.0, -1.0]), np.array([0.8, 0.55]))
    rng = np.random.default_rng(12)
    m.I_bc = rng.uniform(0.0, 0.4, m.F)
    _, dirs, w2 = orc.dirset_uniform(1)
    origins = np.array([6, 25], np.int32)
    J, u = orc.compute_J(m, dirs, w2, origins=origins, want_u=True, dv_max=dv_max, dtau_max=dtau_max)
    checked = 0
    for oi, o in enumerate(origins):
        for r in (0, 3):
            for f in (1, 4, 6):
                ue, gap = _sampled_exact_u(orc.trace_ray, m, int(o), dirs[r], f, m.I_bc[f], dv_max, dtau_max)
                if gap < 1e-9:
                    continue
                assert abs(u[oi, r, f] - float(ue)) <= 1e-12 * abs(float(ue)), (o, r, f)
                checked += 1
    assert checked >= 9


def test_velocity_sampling_converges(orc):
    """A steep velocity gradient along the line: successive halvings of dv_max change J
    less and less."""
    m = synth.tiny_model(53, P=80, F=24, moving=True)
    m.vel = (m.vel * 4.0).astype(np.float32)
    m.freq = synth.FreqGrid(np.array([24], np.int32), np.array([-4.0]), np.array([8.0 / 23]))
    x = m.freq.x()
    m.chi = 0.5 + 5.0 * np.exp(-x[None, :] ** 2) * np.ones((m.P, 1))
    m.eta = m.chi * np.linspace(0.5, 1.5, m.P)[:, None]
    _, dirs, w2 = orc.dirset_uniform(1)
    Js = [orc.compute_J(m, dirs, w2, origins=np.arange(0, m.P, 8), dv_max=v) for v in (1.0, 0.5, 0.25, 0.125)]
    diffs = [np.max(np.abs(Js[i + 1] - Js[i]) / np.abs(Js[-1])) for i in range(3)]
    assert diffs[2] < diffs[0] / 2.5, diffs
