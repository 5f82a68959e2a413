"""Pins of the oracle's HEALPix tables and uniform direction sets (Section 2.1.3, eq. 4)."""
import math

import numpy as np
import pytest


@pytest.mark.parametrize("l", range(0, 6))
def test_npix_is_12_4_l(orc, l):
    # Section 2.1.3: level l has 12 * 4^l pixels.
    assert orc.hp_npix(2 ** l) == 12 * 4 ** l


def test_nside1_closed_form(orc):
    # nside = 1: three rings of four pixels at z = 2/3, 0, -2/3; azimuths
    # pi/4 + k pi/2 on the outer rings and k pi/2 on the equator.
    for p in range(12):
        v = orc.hp_pix2vec(1, p)
        ring, k = divmod(p, 4)
        z = [2.0 / 3.0, 0.0, -2.0 / 3.0][ring]
        phi = (k * math.pi / 2) + (0.0 if ring == 1 else math.pi / 4)
        st = math.sqrt(1 - z * z)
        assert v[2] == pytest.approx(z, abs=1e-15)
        assert v[0] == pytest.approx(st * math.cos(phi), abs=1e-15)
        assert v[1] == pytest.approx(st * math.sin(phi), abs=1e-15)
    # the equatorial pixel 4 is exactly (1, 0, 0)
    assert list(orc.hp_pix2vec(1, 4)) == [1.0, 0.0, 0.0]


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16, 32])
def test_round_trip_and_unit_norm(orc, nside):
    for p in range(orc.hp_npix(nside)):
        v = orc.hp_pix2vec(nside, p)
        assert abs(np.linalg.norm(v) - 1.0) < 4e-16
        assert orc.hp_vec2pix(nside, v) == p


def test_rings_ordered_by_z(orc):
    # ring-scheme indices run from the north pole southwards
    for nside in [2, 4, 8]:
        z = [orc.hp_pix2vec(nside, p)[2] for p in range(orc.hp_npix(nside))]
        assert all(z[i] >= z[i + 1] for i in range(len(z) - 1))
        rings = [orc.hp_ring_of(nside, p) for p in range(orc.hp_npix(nside))]
        assert rings[0] == 1 and rings[-1] == 4 * nside - 1


@pytest.mark.parametrize("nside", [2, 4])
def test_equal_area(orc, nside):
    # Section 2.1.3: pixels of equal area -> isotropic samples fill them uniformly.
    rng = np.random.default_rng(7)
    n = 200_000
    v = rng.normal(size=(n, 3))
    npix = orc.hp_npix(nside)
    h = np.zeros(npix)
    for x in v:
        h[orc.hp_vec2pix(nside, x)] += 1
    e = n / npix
    chi2 = ((h - e) ** 2 / e).sum() / (npix - 1)
    assert 0.7 < chi2 < 1.4


def test_polar_cap_membership_nside1(orc):
    # z > 2/3 lies in the four north base pixels, pixel = azimuth quadrant.
    rng = np.random.default_rng(3)
    for _ in range(2000):
        z = rng.uniform(0.67, 0.999)
        phi = rng.uniform(0, 2 * math.pi)
        st = math.sqrt(1 - z * z)
        v = np.array([st * math.cos(phi), st * math.sin(phi), z])
        assert orc.hp_vec2pix(1, v) == int(phi // (math.pi / 2))
        v[2] = -v[2]
        assert orc.hp_vec2pix(1, v) == 8 + int(phi // (math.pi / 2))


@pytest.mark.parametrize("nside", [2, 4, 8, 16])
def test_hierarchy_four_children(orc, nside):
    # Section 2.1.3: each level-(l-1) pixel is the union of 4 level-l pixels.
    par = [orc.hp_parent(nside, p) for p in range(orc.hp_npix(nside))]
    counts = np.bincount(par, minlength=orc.hp_npix(nside // 2))
    assert np.all(counts == 4)


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
def test_antipode_involution(orc, nside):
    npix = orc.hp_npix(nside)
    a = [orc.hp_antipode(nside, p) for p in range(npix)]
    for p in range(npix):
        assert a[p] != p and a[a[p]] == p
        assert np.allclose(orc.hp_pix2vec(nside, a[p]), -orc.hp_pix2vec(nside, p), atol=1e-15)
        if nside > 1:
            assert orc.hp_parent(nside, a[p]) == orc.hp_antipode(nside // 2, orc.hp_parent(nside, p))


@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_uniform_dirset(orc, nside):
    pix, dirs, w2 = orc.dirset_uniform(nside)
    R = 6 * nside * nside
    assert len(pix) == R and np.all(np.diff(pix) > 0)
    # eq. 4: w = 1/(12 4^l) per ray; the pair weights sum to one
    assert np.all(w2 == 2.0 / (12 * nside * nside))
    assert abs(w2.sum() - 1.0) < 1e-15
    # pairs cover every pixel exactly once with their antipodes
    cover = set(pix.tolist()) | {orc.hp_antipode(nside, int(p)) for p in pix}
    assert cover == set(range(12 * nside * nside))
    # canonical member = smaller index
    assert all(p < orc.hp_antipode(nside, int(p)) for p in pix)
