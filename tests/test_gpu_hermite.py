"""GPU parity of the fourth-order Hermitian rows (Section 2.1: the solver's
fourth-order option with third-order end rows) against the oracle, on the plain
sweep and on refined lines; a step beyond the rows' limit latches RT_ERR_STEP
(and the oracle refuses the same line); a uniform source equal to the incident
intensity is reproduced.

Tolerances.  J, the quantity the method returns: 1e-12 (FP64) and 1e-4 (FP32)
relative, the bars of the second-order path.  The per-pair u (FP64) may also
differ by up to 4 times the oracle's own rounding sensitivity where that is
larger: between very unequal steps a Hermitian weight grows like the step
ratio (1e3 and more on unstructured lines), so a single pair's answer moves by
up to ~1e-12 when the tables move by two ulps, three orders of magnitude more
than the second-order rows' answer does.  The test measures that on the oracle
(its own u under a seeded 2-ulp perturbation of chi and eta) and prints it,
with the same measurement at FP32 size for the record."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-4
HERM = 1
RT_ERR_STEP = -9


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


def _conditioning(orc, m, dirs, w2, oo, c64, e64, kw, u_ref, ulp=2.0 ** -52):
    """Largest relative change of the oracle's u under a 2-ulp perturbation of the tables."""
    rng = np.random.default_rng(1234)
    worst = 0.0
    for _ in range(2):
        cp = c64 * (1.0 + ulp * rng.integers(-2, 3, c64.shape))
        ep = e64 * (1.0 + ulp * rng.integers(-2, 3, e64.shape))
        _, up = orc.compute_J(m, dirs, w2, origins=oo, chi=cp, eta=ep, want_u=True, scheme=HERM, **kw)
        worst = max(worst, _rel(up, u_ref))
    return worst


def _tol64(orc, m, dirs, w2, oo, c64, e64, kw, u_ref):
    k = _conditioning(orc, m, dirs, w2, oo, c64, e64, kw, u_ref)
    tol = max(TOL64, 4.0 * k)
    print(f"oracle conditioning {k:.2e} -> FP64 tolerance {tol:.2e}", flush=True)
    return tol


def _tol32(orc, m, dirs, w2, oo, c64, e64, kw, u_ref):
    """The FP32 kernel forms steps, weights and the elimination in FP32: its answer moves
    like the oracle's under a perturbation of FP32 size, 2^-23 x the 2-ulp FP64 one."""
    k = _conditioning(orc, m, dirs, w2, oo, c64, e64, kw, u_ref, ulp=2.0 ** -23)
    tol = max(TOL32, 4.0 * k)
    print(f"oracle conditioning at FP32 size {k:.2e} -> FP32 tolerance {tol:.2e}", flush=True)
    return tol


def _smooth_sphere():
    """The homogeneous sphere with a source varying smoothly in space: whole steps ~0.2,
    inside the rows' limit, so the plain (unrefined) sweep runs the fourth-order rows."""
    m = synth.sphere_model(F=31)
    r = np.linalg.norm(m.pos, axis=1)
    m.eta = m.chi * (1.0 + 0.5 * np.cos(2.0 * r))[:, None]
    return m


def _case(name):
    if name == "sphere_plain":
        return _smooth_sphere(), 1, {}
    if name == "tiny_moving_dtau":
        m = synth.tiny_model(71, P=60, F=12, moving=True)
        return m, 2, dict(dtau_max=0.5)
    if name == "tiny_2blocks_dtau":  # per-lane Doppler shifts (blocks of different widths)
        m = synth.tiny_model(72, P=50, F=20, moving=True)
        m.freq = synth.FreqGrid(np.array([12, 8], np.int32), np.array([-3.0, -2.0]), np.array([0.5, 0.6]))
        return m, 1, dict(dtau_max=0.4)
    if name == "static_dtau":
        return synth.tiny_model(73, P=50, F=8, moving=False), 2, dict(dtau_max=0.3)
    if name == "tiny_dv_dtau":
        m = synth.tiny_model(74, P=60, F=12, moving=True)
        return m, 2, dict(dv_max=0.25, dtau_max=0.5)
    raise ValueError(name)


@pytest.mark.parametrize("name", ["sphere_plain", "tiny_moving_dtau", "tiny_2blocks_dtau", "static_dtau",
                                  "tiny_dv_dtau"])
def test_hermite_parity_fp64_fp32(rt, orc, name):
    m, nside, kw = _case(name)
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, nside, None)
    Je, ue = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64, want_u=True, scheme=HERM, **kw)
    J2 = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64, **kw)
    assert _rel(J2, Je) > 1e-8  # the scheme changes the answer here
    tol64 = _tol64(orc, m, dirs, w2, oo, c64, e64, kw, ue)
    J64, u64 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F64, c64, e64, want_u=True,
                    scheme=rt.SCHEME_HERMITE, **kw)
    rt.sync_status()
    e_u, e_J = _rel(u64.cpu().numpy(), ue), _rel(J64.cpu().numpy(), Je)
    print(f"{name}: fp64 max rel u {e_u:.2e}, J {e_J:.2e}", flush=True)
    # per-pair u to the oracle's own rounding sensitivity (the rows are that ill-conditioned on some
    # lines); J, the weighted sum over pairs, to the fixed bars of the second-order path
    assert e_u <= tol64
    assert e_J <= TOL64
    _tol32(orc, m, dirs, w2, oo, c64, e64, kw, ue)  # printed for the record
    J32 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F32, c32, e32, scheme=rt.SCHEME_HERMITE, **kw)
    rt.sync_status()
    err = _rel(J32.cpu().numpy().astype(np.float64), Je)
    print(f"{name}: fp32 max rel {err:.2e}", flush=True)
    assert err <= TOL32


def test_hermite_wind_sample(rt, orc):
    """Analytic wind, sampled origins, with optical-depth and velocity refinement keeping
    every step inside the rows' limit."""
    m = synth.wind_model(P=20_000)
    rng = np.random.default_rng(8)
    origins = rng.choice(m.P, 120, replace=False)
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, 2, origins)
    kw = dict(dv_max=1.0 / 3.0, dtau_max=0.5)
    Je, ue = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64, want_u=True, scheme=HERM, **kw)
    _tol64(orc, m, dirs, w2, oo, c64, e64, kw, ue)  # printed for the record
    J64 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F64, c64, e64, scheme=rt.SCHEME_HERMITE, **kw)
    print(f"wind: fp64 max rel J {_rel(J64.cpu().numpy(), Je):.2e}", flush=True)
    assert _rel(J64.cpu().numpy(), Je) <= TOL64
    _tol32(orc, m, dirs, w2, oo, c64, e64, kw, ue)
    J32 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F32, c32, e32, scheme=rt.SCHEME_HERMITE, **kw)
    print(f"wind: fp32 max rel J {_rel(J32.cpu().numpy().astype(np.float64), Je):.2e}", flush=True)
    assert _rel(J32.cpu().numpy().astype(np.float64), Je) <= TOL32
    rt.sync_status()


def test_hermite_uniform_source(rt, orc):
    """S uniform and equal to the incident intensity: J = S to rounding, both precisions.
    S0 is a power of two, so eta = S0 chi holds exactly in each precision's tables and
    after the Doppler interpolation: every S on the line is S0 itself and the right-hand
    sides S0 (1 + E) and S0 carry no rounding; what remains is the elimination's."""
    m = synth.tiny_model(75, P=50, F=12, moving=True)
    S0 = 0.5
    m.eta = m.chi * S0
    m.I_bc = np.full(m.F, S0)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, 2, None)
    J64 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F64, m.chi, m.eta, scheme=rt.SCHEME_HERMITE,
               dtau_max=0.5).cpu().numpy()
    rt.sync_status()
    assert np.max(np.abs(J64 - S0)) < 1e-12
    c32 = m.chi.astype(np.float32)
    J32 = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F32, c32, c32 * np.float32(S0), scheme=rt.SCHEME_HERMITE,
               dtau_max=0.5).cpu().numpy()
    rt.sync_status()
    assert np.max(np.abs(J32 - S0)) < 1e-5


def test_hermite_step_limit_latches_error(rt, orc):
    """Whole steps beyond the limit: the oracle refuses the line and the library latches
    RT_ERR_STEP; the next call starts clean."""
    m = synth.tiny_model(76, P=50, F=12, moving=True)
    m.chi, m.eta = m.chi * 20.0, m.eta * 20.0
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, 2, None)
    with pytest.raises(FloatingPointError):
        orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64, scheme=HERM)
    for prec, (c, e) in ((rt.RT_F64, (c64, e64)), (rt.RT_F32, (c32, e32))):
        with pytest.raises(rt.RtError) as ei:
            _gpu(rt, m, model, ds, rays, org, len(oo), prec, c, e, scheme=rt.SCHEME_HERMITE)
        assert ei.value.code == RT_ERR_STEP
    # the same lines refined below the limit pass, and the word was cleared
    J = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F64, c64, e64, scheme=rt.SCHEME_HERMITE, dtau_max=0.5)
    rt.sync_status()
    assert np.all(np.isfinite(J.cpu().numpy()))


def test_hermite_bad_scheme_rejected(rt):
    m = synth.tiny_model(77, P=30, F=8, moving=False)
    c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    ds = rt.DirSet.uniform(1)
    rays = rt.trace(model, ds)
    with pytest.raises(rt.RtError) as ei:
        _gpu(rt, m, model, ds, rays, None, m.P, rt.RT_F32, c32, e32, scheme=2)
    assert ei.value.code == -1


def test_hermite_plan_graph(rt, orc):
    """Plans carry the scheme: graph replays equal the eager solve."""
    torch = _torch()
    m = _smooth_sphere()
    c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, dirs, w2, oo, org, rays = _setup(rt, orc, m, 1, None)
    ref = _gpu(rt, m, model, ds, rays, org, len(oo), rt.RT_F32, c32, e32, scheme=rt.SCHEME_HERMITE).cpu().numpy()
    J = torch.empty((m.P, m.F), dtype=torch.float32, device="cuda")
    for sched in (rt.SCHED_SPATIAL, rt.SCHED_BINNED):
        plan = rt.Plan(model, ds, _t(c32), _t(e32), m.freq.len, m.freq.dx, _t(m.I_bc, torch.float64), J,
                       origins=org, precision=rt.RT_F32, schedule=sched, scheme=rt.SCHEME_HERMITE)
        for _ in range(2):
            J.zero_()
            plan.run(use_graph=True)
            rt.sync_status()
            assert np.array_equal(J.cpu().numpy(), ref)
        del plan
