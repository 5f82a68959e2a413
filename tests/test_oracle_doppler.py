"""Pin of the oracle's Doppler-shifted optics (Section 2.1.1) by a closed form.

When a point's opacity and emissivity tables are linear in the frequency index
inside each block, chi_q[fb + j] = a + c j, the shifted value the reading
prescribes (the table read at the fractional index j - delta_q, held flat
beyond the block's ends) has the closed form

    chi'_q[f] = a + c clamp(j - delta_q, 0, L - 1),

the straight line evaluated at the clamped continuous coordinate.  This test
builds every line's optics from that closed form in exact rationals (it never
forms interpolation weights or picks table columns), then the trapezoid optical
depths and an exact rational solve of the discrete system, and compares the
oracle's per-pair u.  Because the expected value does not restate the oracle's
interpolation, a swapped (1 - t)/t, an exchanged column pair or a sign error in
delta_q makes the oracle fail it; the second test plants each of those mistakes
in a copy of oracle.c and checks that it does.
"""
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import synth
from exact_feautrier import exact_u

BLOCKS = dict(len=np.array([7, 5], np.int32), x0=np.array([-3.0, -1.0]), dx=np.array([0.6, 0.35]))


def _linear_model(seed=41, P=45):
    """Tiny moving mesh with tables linear in the frequency index inside each block.  The
    coefficients are dyadic (exact in FP64); velocities reach shifts of several block widths,
    so for some points and frequencies the clamp binds fully, for others partly."""
    m = synth.tiny_model(seed, P=P, F=int(BLOCKS["len"].sum()), moving=True)
    m.freq = synth.FreqGrid(BLOCKS["len"].copy(), BLOCKS["x0"].copy(), BLOCKS["dx"].copy())
    rng = np.random.default_rng(seed + 1)
    m.vel = (m.vel * np.float32(0.8)).astype(np.float32)
    F = m.F
    chi = np.zeros((P, F))
    eta = np.zeros((P, F))
    coef = {}
    fb = 0
    for b, L in enumerate(BLOCKS["len"]):
        j = np.arange(L)
        # a in [1, 3], slope in (-a/(L-1), +a) on a 1/64 grid: positive over the block
        a_c = rng.integers(64, 193, P) / 64.0
        s_c = rng.integers(-40, 41, P) / 64.0 * a_c / (L - 1)
        a_e = rng.integers(16, 129, P) / 64.0
        s_e = rng.integers(-60, 61, P) / 64.0 * a_e / (L - 1)
        chi[:, fb:fb + L] = a_c[:, None] + s_c[:, None] * j[None, :]
        eta[:, fb:fb + L] = a_e[:, None] + s_e[:, None] * j[None, :]
        coef[b] = (a_c, s_c, a_e, s_e)
        fb += L
    assert np.all(chi > 0) and np.all(eta > 0)
    m.chi, m.eta = chi, eta
    m.I_bc = rng.uniform(0.0, 0.4, F)
    return m, coef


def _closed_form_u(orc, m, coef, o, d, f):
    """u at origin o, pair direction d, frequency f, from the closed form of the shifted tables."""
    ids_p, Z_p = orc.trace_ray(m, o, d)
    ids_m, Z_m = orc.trace_ray(m, o, -d)
    q = list(ids_m[::-1]) + [o] + list(ids_p)
    s = [-Fr(float(z)) for z in Z_m[::-1]] + [Fr(0)] + [Fr(float(z)) for z in Z_p]
    starts = np.concatenate([[0], np.cumsum(m.freq.len)])
    b = int(np.searchsorted(starts, f, side="right") - 1)
    L, dx = int(m.freq.len[b]), Fr(float(m.freq.dx[b]))
    j = f - int(starts[b])
    a_c, s_c, a_e, s_e = coef[b]
    vo = [Fr(float(v)) for v in m.vel[o]]
    dd = [Fr(float(c)) for c in d]
    chi, S, clamped = [], [], 0
    for p in q:
        delta = sum(a * (Fr(float(v)) - w) for a, v, w in zip(dd, m.vel[p], vo)) / dx
        x = j - delta
        xc = min(max(x, Fr(0)), Fr(L - 1))
        clamped += xc != x
        c = Fr(float(a_c[p])) + Fr(float(s_c[p])) * xc
        e = Fr(float(a_e[p])) + Fr(float(s_e[p])) * xc
        chi.append(c)
        S.append(e / c)
    dtau = [(chi[i] + chi[i + 1]) / 2 * (s[i + 1] - s[i]) for i in range(len(q) - 1)]
    return exact_u(dtau, S, len(ids_m), Fr(float(m.I_bc[f]))), clamped, len(q)


CASES = [(3, 0), (3, 4), (17, 2), (30, 5), (30, 1)]   # (origin, pair of the nside-1 set)
FREQS = (0, 3, 6, 7, 9, 11)                          # both ends and the interior of both blocks


def _check(orc, m, coef, lib_path=None):
    """Largest relative deviation of the oracle's u from the closed form over CASES x FREQS,
    and how many line points had a clamped coordinate."""
    _, dirs, w2 = orc.dirset_uniform(1)
    origins = np.array(sorted({o for o, _ in CASES}), np.int32)
    _, u = orc.compute_J(m, dirs, w2, origins=origins, want_u=True, lib_path=lib_path)
    worst, clamped, points = 0.0, 0, 0
    for o, r in CASES:
        oi = int(np.nonzero(origins == o)[0][0])
        for f in FREQS:
            ue, c, n = _closed_form_u(orc, m, coef, o, dirs[r], f)
            worst = max(worst, abs(u[oi, r, f] - float(ue)) / abs(float(ue)))
            clamped += c
            points += n
    return worst, clamped, points


def test_linear_tables_closed_form(orc):
    m, coef = _linear_model()
    worst, clamped, points = _check(orc, m, coef)
    assert worst <= 1e-12, worst
    # the case exercises the clamp and the unclamped interpolation alike
    assert 0.1 * points < clamped < 0.9 * points, (clamped, points)
    # shifts are generally fractional
    _, dirs, _ = orc.dirset_uniform(1)
    dv = (m.vel - m.vel[3]) @ dirs[0] / m.freq.dx[0]
    assert np.mean(np.abs(dv - np.round(dv)) > 0.05) > 0.5


# (description, text in oracle.c, replacement): plausible mistakes in the shifted optics
PLANTED = [
    ("weights (1-t) and t exchanged",
     "const double xa = (1.0 - t) * ca[ia] + t * ca[ib];\n"
     "                            const double xb = (1.0 - t) * cb[ia] + t * cb[ib];",
     "const double xa = t * ca[ia] + (1.0 - t) * ca[ib];\n"
     "                            const double xb = t * cb[ia] + (1.0 - t) * cb[ib];"),
    ("columns f-k and f-k-1 exchanged",
     "int64_t ia = clampi(j - w.vk[i], 0, L - 1);\n                            int64_t ib = clampi(j - w.vk[i] - 1, 0, L - 1);",
     "int64_t ia = clampi(j - w.vk[i] - 1, 0, L - 1);\n                            int64_t ib = clampi(j - w.vk[i], 0, L - 1);"),
    ("shift with the wrong sign",
     "double delta = w.vdot[i] / blk_dx[b];",
     "double delta = -w.vdot[i] / blk_dx[b];"),
    ("shift in the wrong block's units",
     "double delta = w.vdot[i] / blk_dx[b];",
     "double delta = w.vdot[i] / blk_dx[0];"),
]


@pytest.mark.parametrize("name,old,new", PLANTED, ids=[p[0] for p in PLANTED])
def test_closed_form_catches_planted_mistake(orc, tmp_path, name, old, new):
    src = open(os.path.join(os.path.dirname(orc.__file__), "oracle.c")).read()
    assert src.count(old) == 1, f"planted-mistake anchor not found: {name}"
    path = orc.build_variant(src.replace(old, new), str(tmp_path / "liboracle_variant.so"))
    m, coef = _linear_model()
    worst, _, _ = _check(orc, m, coef, lib_path=path)
    assert worst > 1e-6, f"the closed-form pin did not notice: {name} (worst {worst:.2e})"
