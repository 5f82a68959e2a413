"""GPU parity of the refined lines -- adaptive optical-depth increments (Section
2.1.2, eq. 2) and adaptive velocity sampling (Section 2.1.1) -- against the
oracle: FP64 within 1e-12 and FP32 within 1e-4 relative, split counts decided
identically on both sides; bounds that split nothing leave the sweep
bit-identical to the plain one; the cap on sub-steps is honoured."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-4


def _torch():
    import torch
    return torch


def _t(a, dtype=None):
    torch = _torch()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def _setup(rt, orc, m, nside, origins):
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    ds = rt.DirSet.uniform(nside)
    _, dirs, w2 = orc.dirset_uniform(nside)
    oo = np.arange(m.P, dtype=np.int32) if origins is None else np.asarray(origins, np.int32)
    org = _t(oo)
    rays = rt.trace(model, ds, origins=org)
    return model, ds, dirs, w2, oo, org, rays


def _gpu(rt, m, model, ds, rays, org, n_o, prec, chi, eta, **kw):
    torch = _torch()
    dt = np.float64 if prec == rt.RT_F64 else np.float32
    return rt.solve(model, ds, rays, _t(chi.astype(dt)), _t(eta.astype(dt)), m.freq.len, m.freq.dx,
                    _t(m.I_bc, torch.float64), origins=org, n_origins=n_o, precision=prec, **kw)


@pytest.mark.parametrize("case,dtau_max", [("tiny_moving", 0.15), ("tiny_2blocks", 0.1), ("static", 0.05),
                                           ("sphere", 0.2)])
def test_substep_parity_fp64_fp32(rt, orc, case, dtau_max):
    if case == "tiny_moving":
        m, nside = synth.tiny_model(41, P=60, F=12, moving=True), 2
        m.chi, m.eta = m.chi * 3.0, m.eta * 3.0
    elif case == "tiny_2blocks":  # per-lane Doppler shifts (blocks of different widths)
        m, nside = synth.tiny_model(42, P=50, F=20, moving=True), 1
        m.freq = synth.FreqGrid(np.array([12, 8], np.int32), np.array([-3.0, -2.0]), np.array([0.5, 0.6]))
        m.chi, m.eta = m.chi * 2.0, m.eta * 2.0
    elif case == "static":
        m, nside = synth.tiny_model(43, P=50, F=8, moving=False), 2
    else:
        m, nside = synth.sphere_model(), 1
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, nside, None)
    Je, ue = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64, want_u=True, dtau_max=dtau_max)
    J0 = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64)
    assert _rel(J0, Je) > 1e-6  # the bound does split intervals here
    J64, u64 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F64, c64, e64, dtau_max=dtau_max, want_u=True)
    rt.sync_status()
    assert _rel(u64.cpu().numpy(), ue) <= TOL64
    assert _rel(J64.cpu().numpy(), Je) <= TOL64
    J32 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F32, c32, e32, dtau_max=dtau_max)
    err = _rel(J32.cpu().numpy().astype(np.float64), Je)
    print(f"{case}: fp32 max rel {err:.2e}")
    assert err <= TOL32


def test_substep_wind_sample(rt, orc):
    """The analytic wind: line centres are optically thick near the inner edge."""
    m = synth.wind_model(P=20_000)
    rng = np.random.default_rng(3)
    origins = rng.choice(m.P, 150, replace=False)
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, 2, origins)
    Je = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64, dtau_max=0.1)
    J64 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F64, c64, e64, dtau_max=0.1)
    assert _rel(J64.cpu().numpy(), Je) <= TOL64
    J32 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F32, c32, e32, dtau_max=0.1)
    assert _rel(J32.cpu().numpy().astype(np.float64), Je) <= TOL32
    rt.sync_status()


def test_large_bound_is_bit_identical(rt, orc):
    m = synth.tiny_model(44, P=60, F=16, moving=True)
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, 2, None)
    for prec, (c, e) in ((rt.RT_F64, (c64, e64)), (rt.RT_F32, (c32, e32))):
        J0 = _gpu(rt, m, model, ds, rays, org, len(oo), prec, c, e).cpu().numpy()
        J1 = _gpu(rt, m, model, ds, rays, org, len(oo), prec, c, e, dtau_max=1e9).cpu().numpy()
        assert np.array_equal(J0, J1)


def test_substep_cap(rt, orc):
    m = synth.tiny_model(45, P=40, F=8, moving=True)
    m.chi, m.eta = m.chi * 20.0, m.eta * 20.0
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, 1, None)
    Je = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64, dtau_max=1e-3, max_sub=3)
    J64 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F64, c64, e64, dtau_max=1e-3, max_substeps=3)
    assert _rel(J64.cpu().numpy(), Je) <= TOL64


def test_substep_plan_graph(rt, orc):
    """Plans carry the option: graph replays equal the eager solve with the same bound."""
    torch = _torch()
    m = synth.tiny_model(46, P=80, F=16, moving=True)
    m.chi, m.eta = m.chi * 3.0, m.eta * 3.0
    c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, 2, None)
    ref = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F32, c32, e32, dtau_max=0.2).cpu().numpy()
    J = torch.empty((m.P, m.F), dtype=torch.float32, device="cuda")
    plan = rt.Plan(model, ds, _t(c32), _t(e32), m.freq.len, m.freq.dx, _t(m.I_bc, torch.float64), J,
                   origins=org, precision=rt.RT_F32, schedule=rt.SCHED_SPATIAL, dtau_max=0.2)
    for _ in range(2):
        J.zero_()
        plan.run(use_graph=True)
        rt.sync_status()
        assert np.array_equal(J.cpu().numpy(), ref)


# ----------------------------------------------------------------------------- velocity sampling (Section 2.1.1)

@pytest.mark.parametrize("case,dv_max,dtau_max", [("tiny", 0.3, 0.0), ("tiny", 0.25, 0.2),
                                                  ("two_blocks", 0.4, 0.0), ("two_blocks", 0.2, 0.15)])
def test_velocity_sampling_parity(rt, orc, case, dv_max, dtau_max):
    if case == "tiny":
        m, nside = synth.tiny_model(61, P=60, F=12, moving=True), 2
        m.chi, m.eta = m.chi * 2.0, m.eta * 2.0
    else:  # per-lane shifts: blocks of different widths
        m, nside = synth.tiny_model(62, P=50, F=20, moving=True), 1
        m.freq = synth.FreqGrid(np.array([12, 8], np.int32), np.array([-3.0, -2.0]), np.array([0.5, 0.6]))
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, nside, None)
    Je, ue = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64, want_u=True, dv_max=dv_max,
                           dtau_max=dtau_max)
    assert _rel(orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64, dtau_max=dtau_max), Je) > 1e-6
    J64, u64 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F64, c64, e64, dv_max=dv_max, dtau_max=dtau_max,
                    want_u=True)
    rt.sync_status()
    assert _rel(u64.cpu().numpy(), ue) <= TOL64
    J32 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F32, c32, e32, dv_max=dv_max, dtau_max=dtau_max)
    err = _rel(J32.cpu().numpy().astype(np.float64), Je)
    print(f"{case} dv {dv_max} dtau {dtau_max}: fp32 max rel {err:.2e}")
    assert err <= TOL32


def test_velocity_sampling_wind(rt, orc):
    """The wind's radial flow reaches 20 Doppler widths: rays crossing it get sampled."""
    m = synth.wind_model(P=20_000)
    rng = np.random.default_rng(4)
    origins = rng.choice(m.P, 120, replace=False)
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, 2, origins)
    Je = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64, dv_max=1.0 / 3.0, dtau_max=0.5)
    J64 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F64, c64, e64, dv_max=1.0 / 3.0, dtau_max=0.5)
    assert _rel(J64.cpu().numpy(), Je) <= TOL64
    J32 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F32, c32, e32, dv_max=1.0 / 3.0, dtau_max=0.5)
    assert _rel(J32.cpu().numpy().astype(np.float64), Je) <= TOL32
    rt.sync_status()


def test_refined_path_without_splits_is_bit_identical(rt, orc):
    """Bounds that split nothing: the refined sweep gives the plain sweep's bits."""
    for seed, blocks in ((63, False), (64, True)):
        m = synth.tiny_model(seed, P=50, F=12, moving=True)
        if blocks:
            m.freq = synth.FreqGrid(np.array([7, 5], np.int32), np.array([-3.0, -1.0]), np.array([0.5, 0.7]))
        c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
        model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, 2, None)
        for prec, (c, e) in ((rt.RT_F64, (c64, e64)), (rt.RT_F32, (c32, e32))):
            J0 = _gpu(rt, m, model, ds, rays, org, len(oo), prec, c, e).cpu().numpy()
            J1 = _gpu(rt, m, model, ds, rays, org, len(oo), prec, c, e, dv_max=1e9, dtau_max=1e9).cpu().numpy()
            assert np.array_equal(J0, J1)
