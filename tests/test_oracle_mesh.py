"""Pins of the re-meshing indicators (Section 2.2.2, eqs. 6-8, Table 1)."""
import numpy as np

import synth
from oracle import mesh as om


def test_lattice_sizes_and_uniform_tracer():
    m = synth.lattice_model(5, F=1, spacing=0.25)  # face neighbours: every distance is the spacing
    Gf, L, ell = om.mesh_indicators(m, np.full(m.P, 3.0), *om.TABLE1["AMR"])
    assert np.all(L == 0.25) and np.all(Gf == 0.0)
    assert np.allclose(ell, 0.25 * 2.10)          # no change anywhere: coarsen everywhere


def test_two_valued_tracer():
    """A step between two values a, b: Gf = |a-b|/(a+b) exactly at the points touching the
    other value, 0 elsewhere; the threshold picks f_small there."""
    m = synth.lattice_model(6, F=1)
    x = m.pos[:, 0]
    a, b = 1.0, 3.0
    f = np.where(x < 2.5, a, b)
    Gf, L, ell = om.mesh_indicators(m, f, *om.TABLE1["SPH"])
    edge = (x == 2.0) | (x == 3.0)
    assert np.allclose(Gf[edge], 0.5) and np.all(Gf[~edge] == 0.0)
    assert np.allclose(ell[edge], L[edge] * 1.00) and np.allclose(ell[~edge], L[~edge] * 2.15)


def test_bounds_and_symmetry():
    m = synth.tiny_model(7, P=80, F=1)
    rng = np.random.default_rng(1)
    f = 10.0 ** rng.uniform(-3, 3, m.P)
    Gf, L, _ = om.mesh_indicators(m, f, *om.TABLE1["AMR"])
    assert np.all((0 <= Gf) & (Gf < 1))
    # scaling the tracer changes nothing (Gf is a ratio); a point's L is its mean edge length
    Gf2, _, _ = om.mesh_indicators(m, 7.5 * f, *om.TABLE1["AMR"])
    assert np.allclose(Gf, Gf2, rtol=1e-14, atol=1e-16)
    i = 11
    nb = m.nbr_idx[m.nbr_off[i]:m.nbr_off[i + 1]]
    assert np.isclose(L[i], sum(np.linalg.norm(m.pos[i] - m.pos[n]) for n in nb) / len(nb))


def _golden_table1():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_reduction_parameters.txt")
    rows = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            name, *vals = line.split()
            rows[name] = tuple(float(v) for v in vals)
    return rows


def test_table1_constants_are_the_papers():
    """The oracle's and the library's reduction parameters equal the values the
    paper prints in Table 1 (stored fixture)."""
    import paper_2011_14998_amd.binding as b
    t = _golden_table1()
    assert set(t) == {"AMR", "SPH"}
    for k, v in t.items():
        assert tuple(om.TABLE1[k]) == v
        assert tuple(b.REDUCTION_PARAMS[k]) == v
