"""GPU parity of the re-meshing indicators (eqs. 6-8) against the oracle:
Gf bit for bit (one IEEE division per neighbour, the same maximum), L within
1e-14, and the size map taking the same threshold decisions."""
import numpy as np
import pytest

import synth
from oracle import mesh as om

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["octree", "sph", "lattice"])
def test_mesh_indicators(rt, case):
    import torch
    if case == "octree":
        m, params = synth.octree_model(seed=3, target=60_000), om.TABLE1["AMR"]
        f = (m.chi[:, 0] / m.chi[:, 0].max()) ** 0.15  # a smoother tracer: both branches occur
    elif case == "sph":
        m, params = synth.sph_cloud_model(seed=401, P=15_000), om.TABLE1["SPH"]
        f = m.chi[:, 0]
    else:
        m, params = synth.lattice_model(8, F=1), om.TABLE1["AMR"]
        f = np.where(m.pos[:, 2] < 3.5, 1.0, 1.5)
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, None)
    Gf, L, ell = rt.mesh_indicators(model, torch.as_tensor(np.ascontiguousarray(f, np.float64), device="cuda"),
                                    *params)
    eG, eL, eell = om.mesh_indicators(m, f, *params)
    Gf, L, ell = Gf.cpu().numpy(), L.cpu().numpy(), ell.cpu().numpy()
    assert np.array_equal(Gf, eG)
    assert np.max(np.abs(L - eL) / eL) <= 1e-14
    # the same branch at every point (the products differ only in the last bit of L)
    small = np.isclose(ell / L, params[0], rtol=1e-12, atol=0)
    assert np.array_equal(small, np.isclose(eell / eL, params[0], rtol=1e-12, atol=0))
    assert np.array_equal(small, eG >= params[2]) or params[0] == params[1]
    assert np.max(np.abs(ell - eell) / eell) <= 1e-14
    frac = np.mean(Gf >= params[2])
    print(f"{case}: {m.P} points, {frac:.3f} above the threshold")
