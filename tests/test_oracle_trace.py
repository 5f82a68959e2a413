"""Pins of the oracle's ray tracer (Section 2.1, Fig. 2: point-to-point stepping
along a straight line; each step goes to the forward neighbour closest to the
ray axis, the distance increment being the projection of the Delaunay edge)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.spatial as sps

import synth


def _exact_trace(pos, off, idx, o, d):
    """The stepping rule evaluated in exact rational arithmetic on the FP64 inputs.

    Returns (ids, Z_exact, near_tie): near_tie is True when some decision was
    within 1e-12 (relative) of flipping, where FP64 may legitimately differ."""
    Fr = Fraction
    dd = [Fr(float(x)) for x in d]
    xo = [Fr(float(x)) for x in pos[o]]
    c, Zc = o, Fr(0)
    ids, Zs, near = [], [], False
    for _ in range(len(pos)):
        cands = []
        for e in range(off[c], off[c + 1]):
            k = int(idx[e])
            R = [Fr(float(pos[k][i])) - xo[i] for i in range(3)]
            Z = R[0] * dd[0] + R[1] * dd[1] + R[2] * dd[2]
            scale = abs(R[0]) + abs(R[1]) + abs(R[2])
            if abs(Z - Zc) <= Fr(1, 10 ** 12) * scale:
                near = True
            if Z <= Zc:
                continue
            q = [R[i] - Z * dd[i] for i in range(3)]
            D = q[0] * q[0] + q[1] * q[1] + q[2] * q[2]
            cands.append((D, k, Z, scale))
        if not cands:
            break
        cands.sort(key=lambda t: (t[0], t[1]))
        if len(cands) > 1 and cands[1][0] - cands[0][0] <= Fr(1, 10 ** 12) * cands[0][3] ** 2:
            near = True
        D, k, Z, _ = cands[0]
        ids.append(k)
        Zs.append(Z)
        c, Zc = k, Z
    return ids, Zs, near


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_exact_rational_bruteforce(orc, seed):
    m = synth.tiny_model(seed, P=45)
    _, dirs, _ = orc.dirset_uniform(1)
    checked = 0
    for o in range(m.P):
        for r in range(len(dirs)):
            for sgn in (1.0, -1.0):
                d = dirs[r] * sgn
                ids, Z = orc.trace_ray(m, o, d)
                eids, eZ, near = _exact_trace(m.pos, m.nbr_off, m.nbr_idx, o, d)
                if near:
                    continue
                checked += 1
                assert list(ids) == eids
                for z, ez in zip(Z, eZ):
                    assert abs(Fraction(float(z)) - ez) <= Fraction(1, 10 ** 14) * (abs(ez) + 1)
    assert checked > 0.9 * m.P * 12


def _rnd(x):
    """Round an exact rational to the nearest FP64 (ties to even)."""
    return Fraction(x.numerator / x.denominator) if x.denominator != 1 else Fraction(float(x.numerator))


def test_recorded_Z_is_the_stated_fma_chain(orc):
    """The recorded projection of each step is the stated FP64 evaluation:
    R = x_k - x_o rounded per axis, then Z = fma(R.z, d.z, fma(R.y, d.y, R.x d.x)),
    each operation rounded once (evaluated here in exact rationals)."""
    m = synth.tiny_model(14, P=40)
    _, dirs, _ = orc.dirset_uniform(1)
    n = 0
    for o in range(0, m.P, 3):
        for r in range(len(dirs)):
            for sgn in (1.0, -1.0):
                d = [Fraction(float(x)) for x in dirs[r] * sgn]
                ids, Z = orc.trace_ray(m, o, dirs[r] * sgn)
                for k, z in zip(ids, Z):
                    R = [_rnd(Fraction(float(m.pos[k][i])) - Fraction(float(m.pos[o][i]))) for i in range(3)]
                    e = _rnd(R[0] * d[0])
                    e = _rnd(R[1] * d[1] + e)
                    e = _rnd(R[2] * d[2] + e)
                    assert Fraction(float(z)) == e
                    n += 1
    assert n > 100


def _forward_set(m, c, o, d, Zc):
    ks = m.nbr_idx[m.nbr_off[c]:m.nbr_off[c + 1]]
    R = m.pos[ks] - m.pos[o]
    Z = R @ d
    return ks[Z > Zc], R[Z > Zc], Z[Z > Zc]


@pytest.mark.parametrize("seed", [21, 22])
def test_invariants_and_hull_termination(orc, seed):
    m = synth.tiny_model(seed, P=60)
    hull = set(sps.ConvexHull(m.pos).vertices.tolist())
    _, dirs, _ = orc.dirset_uniform(2)
    for o in range(0, m.P, 3):
        for d0 in dirs:
            for d in (d0, -d0):
                ids, Z = orc.trace_ray(m, o, d)
                prev, Zc = o, 0.0
                for k, z in zip(ids, Z):
                    # consecutive points are neighbours, Z strictly increases
                    assert k in m.nbr_idx[m.nbr_off[prev]:m.nbr_off[prev + 1]]
                    assert z > Zc
                    # the chosen point minimises the distance to the axis, computed
                    # here independently as |R x d|^2 over the forward set
                    ks, R, _ = _forward_set(m, prev, o, d, Zc)
                    dist = np.sum(np.cross(R, d) ** 2, axis=1)
                    assert dist[list(ks).index(k)] <= dist.min() * (1 + 1e-9) + 1e-300
                    prev, Zc = k, z
                # the ray stops only where no neighbour lies ahead, which in a
                # Delaunay mesh happens only on the convex hull
                ks, _, _ = _forward_set(m, prev, o, d, Zc)
                assert len(ks) == 0
                assert prev in hull


def test_lattice_axis_rays(orc):
    n = 6
    m = synth.lattice_model(n)
    lin = lambda i, j, k: (i * n + j) * n + k  # noqa: E731
    o = lin(1, 2, 3)
    ids, Z = orc.trace_ray(m, o, np.array([1.0, 0.0, 0.0]))
    assert list(ids) == [lin(i, 2, 3) for i in range(2, n)]
    assert list(Z) == [1.0, 2.0, 3.0, 4.0]
    ids, Z = orc.trace_ray(m, o, np.array([-1.0, -0.0, -0.0]))
    assert list(ids) == [lin(0, 2, 3)] and list(Z) == [1.0]
    ids, Z = orc.trace_ray(m, o, np.array([0.0, 0.0, 1.0]))
    assert list(ids) == [lin(1, 2, 4), lin(1, 2, 5)]
    # the nside = 1 equatorial pixel 4 is exactly +x
    _, dirs, _ = orc.dirset_uniform(1)
    ids2, _ = orc.trace_ray(m, o, dirs[4])
    assert list(ids2) == [lin(i, 2, 3) for i in range(2, n)]


def test_trace_all_layout(orc):
    m = synth.tiny_model(5, P=30)
    _, dirs, _ = orc.dirset_uniform(1)
    origins = np.array([3, 7, 11], np.int32)
    off, ids, Z = orc.trace_all(m, dirs, origins)
    R = len(dirs)
    assert len(off) == len(origins) * 2 * R + 1
    for oi, o in enumerate(origins):
        for r in range(R):
            for s, sgn in ((0, 1.0), (1, -1.0)):
                slot = oi * 2 * R + 2 * r + s
                a, b = off[slot], off[slot + 1]
                e_ids, e_Z = orc.trace_ray(m, int(o), dirs[r] * sgn)
                assert list(ids[a:b]) == list(e_ids)
                assert np.array_equal(Z[a:b], e_Z)


def test_sphere_rays_end_on_boundary(orc):
    m = synth.sphere_model()
    _, dirs, _ = orc.dirset_uniform(2)
    off, ids, _ = orc.trace_all(m, dirs, np.arange(m.P, dtype=np.int32))
    lens = np.diff(off)
    ends = ids[off[1:][lens > 0] - 1]
    hull = set(sps.ConvexHull(m.pos).vertices.tolist())
    assert set(ends.tolist()) <= hull
    # points inside the hull always have a forward neighbour, in every direction
    inner = np.array([p not in hull for p in range(m.P)])
    assert inner.sum() > 900
    assert np.all(lens.reshape(m.P, -1)[inner] > 0)
