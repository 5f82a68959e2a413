"""Pins of the oracle's adaptive direction sets (Section 2.1.3, Fig. 1)."""
import math

import numpy as np
import pytest

import synth


def test_fixed_sqrt_and_atan2_match_libm(orc):
    rng = np.random.default_rng(0)
    for x in 10.0 ** rng.uniform(-300, 300, 5000):
        assert abs(orc.fx_sqrt(x) - math.sqrt(x)) <= 2.3e-16 * math.sqrt(x)
    for y, x in rng.normal(size=(5000, 2)):
        assert abs(orc.fx_atan2(y, x) - math.atan2(y, x)) <= 9e-16
    for y, x in ((0.0, 1.0), (1.0, 0.0), (0.0, -1.0), (-1.0, 0.0), (1.0, 1.0), (-3.0, -3.0)):
        assert abs(orc.fx_atan2(y, x) - math.atan2(y, x)) <= 4.5e-16


def test_fixed_lookup_equals_library_lookup(orc):
    rng = np.random.default_rng(1)
    for nside in (1, 2, 8, 16):
        diff = 0
        for v in rng.normal(size=(4000, 3)):
            diff += orc.fx_vec2pix(nside, v) != orc.hp_vec2pix(nside, v)
        assert diff <= 1  # only directions within ~1e-15 of a pixel boundary may differ


@pytest.mark.parametrize("lmin,lmax,rays", [(1, 4, 552), (0, 3, 138), (2, 2, 192), (1, 2, 120)])
def test_ray_counts(orc, lmin, lmax, rays):
    # Section 3.2.1: 552 rays for l = 1 .. 4; the same number for every point
    assert 2 * orc.dirset_adaptive_R(lmin, lmax) == rays


def _py_vec2pix(nside, v):
    """Textbook ring-scheme lookup with numpy's arctan2 (independent of the oracle)."""
    x, y, z = v / np.linalg.norm(v)
    phi = math.atan2(y, x) % (2 * math.pi)
    za, tt = abs(z), phi / (math.pi / 2)
    ncap, npix = 2 * nside * (nside - 1), 12 * nside * nside
    if za <= 2 / 3:
        jp = int(math.floor(nside * (0.5 + tt) - 0.75 * nside * z))
        jm = int(math.floor(nside * (0.5 + tt) + 0.75 * nside * z))
        ir = nside + 1 + jp - jm
        ip = ((jp + jm - nside + (1 - (ir & 1)) + 1) // 2) % (4 * nside)
        return ncap + (ir - 1) * 4 * nside + ip
    tp = tt - math.floor(tt)
    tmp = nside * math.sqrt(3 * (1 - za))
    jp, jm = int(math.floor(tp * tmp)), int(math.floor((1 - tp) * tmp))
    ir = jp + jm + 1
    ip = int(math.floor(tt * ir)) % (4 * ir)
    return 2 * ir * (ir - 1) + ip if z > 0 else npix - 2 * ir * (ir + 1) + ip


def _py_adaptive(orc, pos, o, sample, lmin, lmax):
    """Brute-force restatement: histogram, downgrade, top-half refinement, sorted leaves."""
    L = lmax - lmin + 1
    ns = [2 ** (lmin + k) for k in range(L)]
    cen = [[orc.hp_pix2vec(n, p) for p in range(12 * n * n)] for n in ns]
    anti = [[_py_vec2pix(n, -c) for c in cen[k]] for k, n in enumerate(ns)]
    par = [None] + [[_py_vec2pix(ns[k - 1], c) for c in cen[k]] for k in range(1, L)]
    h = [np.zeros(12 * n * n, np.int64) for n in ns]
    near = False
    for s in sample:
        v = pos[s] - pos[o]
        if s == o or not v.any():
            continue
        p = _py_vec2pix(ns[-1], v)
        # a direction within 1e-10 of a boundary may legitimately classify differently
        for eps in (1e-10, -1e-10):
            if _py_vec2pix(ns[-1], v + eps * np.array([0.37, -0.61, 0.7])) != p:
                near = True
        h[-1][p] += 1
    for k in range(L - 1, 0, -1):
        for p in range(len(h[k])):
            h[k - 1][par[k][p]] += h[k][p]
    cnt = lambda k, p: h[k][p] + h[k][anti[k][p]]  # noqa: E731
    act = [p for p in range(len(h[0])) if anti[0][p] > p]
    leaves = []
    for k in range(L):
        if k == L - 1:
            leaves += [(lmin + k, p) for p in act]
            break
        act.sort(key=lambda p: (-cnt(k, p), p))
        half = len(act) // 2
        leaves += [(lmin + k, p) for p in act[half:]]
        ref = set(act[:half])
        act = sorted({min(c, anti[k + 1][c]) for c in range(len(h[k + 1])) if par[k + 1][c] in ref})
    return sorted(leaves), near


@pytest.mark.parametrize("seed", [3, 4])
def test_bruteforce_small(orc, seed):
    m = synth.tiny_model(seed, P=50)
    rng = np.random.default_rng(seed)
    sample = rng.choice(m.P, 40, replace=False).astype(np.int32)
    pix, lev, dirs, w2 = orc.dirset_adaptive(m, 1, 3, sample, origins=np.arange(m.P))
    checked = 0
    for o in range(m.P):
        exp, near = _py_adaptive(orc, m.pos, o, sample, 1, 3)
        if near:
            continue
        checked += 1
        assert list(zip(lev[o].tolist(), pix[o].tolist())) == exp
    assert checked >= 40


def test_weights_partition_and_lmax_identity(orc):
    m = synth.wind_model(P=3000)
    rng = np.random.default_rng(5)
    sample = rng.choice(m.P, 1000, replace=False).astype(np.int32)
    origins = np.arange(0, m.P, 37)
    pix, lev, dirs, w2 = orc.dirset_adaptive(m, 1, 4, sample, origins=origins)
    assert np.allclose(w2.sum(1), 1.0, rtol=0, atol=1e-15)
    upix, udirs, _ = orc.dirset_uniform(16)
    where = {int(p): i for i, p in enumerate(upix)}
    for o in range(len(origins)):
        # every level-4 pixel has exactly one ancestor-or-self among the leaves and their antipodes
        cover = np.zeros(12 * 16 * 16, int)
        for l, p in zip(lev[o], pix[o]):
            for q in (int(p), orc.hp_antipode(2 ** int(l), int(p))):
                for f in range(12 * 16 * 16):
                    g, lf = f, 4
                    while lf > l:
                        g = orc.hp_parent(2 ** lf, g)
                        lf -= 1
                    if g == q:
                        cover[f] += 1
        assert np.all(cover == 1)
        # Section 3.2.1: maximally refined directions are exactly the dense regular ones
        for l, p, d in zip(lev[o], pix[o], dirs[o]):
            if l == 4:
                assert np.array_equal(d, udirs[where[int(p)]])
        if o >= 2:
            break


def test_refinement_follows_point_density(orc):
    # all sample points in one direction: the pairs around it are refined to lmax
    pos = np.zeros((200, 3))
    rng = np.random.default_rng(6)
    pos[1:] = np.array([0.1, 0.2, 5.0]) + 0.05 * rng.normal(size=(199, 3))
    m = synth.Model("cone", pos, np.zeros(201, np.int64), np.zeros(0, np.int32), None, np.ones((200, 1)),
                    np.ones((200, 1)), synth.FreqGrid.uniform(1, 1), np.zeros(1))
    pix, lev, dirs, w2 = orc.dirset_adaptive(m, 1, 4, np.arange(200, dtype=np.int32), origins=[0])
    up = dirs[0][lev[0] == 4]
    # the finest pairs point (up to sign) towards +z where the points are
    assert np.max(np.abs(up @ np.array([0.0, 0.0, 1.0]))) > 0.99


def test_empty_sample_refines_lowest_indices(orc):
    m = synth.tiny_model(7, P=20)
    pix, lev, dirs, w2 = orc.dirset_adaptive(m, 1, 2, np.zeros(0, np.int32), origins=[0])
    _, _, _ = orc.dirset_uniform(2)
    lv1 = sorted(pix[0][lev[0] == 1].tolist())
    canon1 = [p for p in range(48) if orc.hp_antipode(2, p) > p]
    assert lv1 == canon1[12:]  # counts all zero: the 12 smallest indices are refined


def test_ray_counts_printed_in_the_paper(orc):
    """The stored fixture holds the ray counts the paper prints (Section 3.2.1):
    the oracle's regular and adaptive sets have exactly those."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "ray_counts.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for kind, lmin, lmax, rays in rows:
        lmin, lmax, rays = int(lmin), int(lmax), int(rays)
        if kind == "regular":
            _, dirs, w2 = orc.dirset_uniform(2 ** lmax)
            assert 2 * len(dirs) == rays
            # eq. 4: each ray weighs 1/(12 4^l); a pair carries both rays' weight
            assert np.all(w2 == 2.0 / rays)
        else:
            assert 2 * orc.dirset_adaptive_R(lmin, lmax) == rays
