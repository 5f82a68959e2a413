"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Bars: ray lists (ids and Z) bit-exact; J within 1e-12 relative on the FP64 path
and within 1e-4 relative on the FP32 sweep (both against the FP64 oracle fed the
same table values); schedules and graph replays bit-identical to each other.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-4


def _torch():
    import torch
    return torch


def _gpu_model(rt, m):
    return rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)


def _t(a, dtype=None):
    torch = _torch()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _trace_both(rt, orc, m, nside, origins):
    model = _gpu_model(rt, m)
    ds = rt.DirSet.uniform(nside)
    _, dirs, w2 = orc.dirset_uniform(nside)
    org = None if origins is None else _t(origins.astype(np.int32))
    n_o = m.P if origins is None else len(origins)
    off, ids, Z = rt.trace(model, ds, origins=org, n_origins=n_o)
    oo = np.arange(m.P, dtype=np.int32) if origins is None else origins.astype(np.int32)
    e_off, e_ids, e_Z = orc.trace_all(m, dirs, oo)
    return model, ds, (off, ids, Z), (e_off, e_ids, e_Z), dirs, w2, org, oo


def _assert_rays_equal(g, e):
    off, ids, Z = (x.cpu().numpy() for x in g)
    assert np.array_equal(off, e[0])
    assert np.array_equal(ids, e[1])
    assert np.array_equal(Z.view(np.uint64), e[2].view(np.uint64))


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


# ----------------------------------------------------------------------------- tracing

@pytest.mark.parametrize("nside", [1, 2])
def test_trace_sphere_all_origins(rt, orc, nside):
    m = synth.sphere_model()
    _, _, g, e, *_ = _trace_both(rt, orc, m, nside, None)
    _assert_rays_equal(g, e)


def test_trace_lattice_ties(rt, orc):
    # exact distance ties and the exact +x direction at nside 1
    m = synth.lattice_model(7)
    _, _, g, e, *_ = _trace_both(rt, orc, m, 1, np.arange(m.P))
    _assert_rays_equal(g, e)


def test_trace_ties_independent_of_row_order(rt, orc):
    """Each point's neighbours in a seeded random order: on the lattice (exact
    distance ties everywhere) the lists equal the oracle's on the original order."""
    m = synth.lattice_model(6)
    rng = np.random.default_rng(17)
    idx = m.nbr_idx.copy()
    for p in range(m.P):
        a, b = m.nbr_off[p], m.nbr_off[p + 1]
        idx[a:b] = idx[a:b][rng.permutation(b - a)]
    assert not np.array_equal(idx, m.nbr_idx)
    shuffled = synth.Model(m.name, m.pos, m.nbr_off, idx, m.vel, m.chi, m.eta, m.freq, m.I_bc)
    model = _gpu_model(rt, shuffled)
    ds = rt.DirSet.uniform(1)
    off, ids, Z = rt.trace(model, ds)
    _, dirs, _ = orc.dirset_uniform(1)
    e_off, e_ids, e_Z = orc.trace_all(m, dirs, np.arange(m.P, dtype=np.int32))
    _assert_rays_equal((off, ids, Z), (e_off, e_ids, e_Z))


def test_model_rejects_huge_positions(rt):
    m = synth.tiny_model(6, P=20)
    pos = m.pos.copy()
    pos[3, 1] = 1e200
    with pytest.raises(rt.RtError) as ex:
        rt.Model.from_numpy(pos, m.nbr_off, m.nbr_idx)
    assert ex.value.code == -1


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_trace_tiny(rt, orc, seed):
    m = synth.tiny_model(seed, P=60)
    _, _, g, e, *_ = _trace_both(rt, orc, m, 4, None)
    _assert_rays_equal(g, e)


@pytest.mark.parametrize("nside,n_org", [(2, 3000), (4, 700)])
def test_trace_wind_sampled(rt, orc, wind, nside, n_org):
    rng = np.random.default_rng(nside)
    origins = rng.choice(wind.P, n_org, replace=False)
    _, _, g, e, *_ = _trace_both(rt, orc, wind, nside, origins)
    _assert_rays_equal(g, e)


def test_trace_degenerate_meshes(rt, orc):
    # two points, three collinear points: lines of length 1..3, empty rays
    for pos in (np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]]),
                np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [2.0, 0.0, 0.0]])):
        P = len(pos)
        a = np.arange(P - 1)
        off, idx = synth.models.csr_from_edges(P, a, a + 1)
        m = synth.Model("line", pos, off, idx, None, np.ones((P, 3)), np.ones((P, 3)) * 0.5,
                        synth.FreqGrid.uniform(1, 3), np.zeros(3))
        _, _, g, e, *_ = _trace_both(rt, orc, m, 1, None)
        _assert_rays_equal(g, e)


def test_trace_capacity_error_is_reported(rt):
    import ctypes as C
    torch = _torch()
    m = synth.tiny_model(4, P=30)
    model = _gpu_model(rt, m)
    ds = rt.DirSet.uniform(1)
    off, ids, Z = rt.trace(model, ds)
    total = ids.numel()
    small = total // 2
    ids2 = torch.empty(small, dtype=torch.int32, device="cuda")
    Z2 = torch.empty(small, dtype=torch.float64, device="cuda")
    L = rt.binding.load()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.rt_trace_write(model._h, ds._h, None, m.P, off.data_ptr(), ids2.data_ptr(), Z2.data_ptr(), small, s) == 0
    with pytest.raises(rt.RtError) as ex:
        rt.sync_status()
    assert ex.value.code == -4
    rt.sync_status()  # cleared


def test_model_rejects_bad_indices(rt):
    m = synth.tiny_model(5, P=20)
    idx = m.nbr_idx.copy()
    idx[7] = 1000
    with pytest.raises(rt.RtError) as ex:
        rt.Model.from_numpy(m.pos, m.nbr_off, idx)
    assert ex.value.code == -2


@pytest.mark.parametrize("case", ["non_monotone", "short_end", "self_neighbour", "negative_index"])
def test_model_rejects_bad_csr(rt, case):
    """A malformed CSR is refused by the check that runs before the records are laid out
    (the layout scans the degrees, so it only ever sees offsets that run from 0 to E)."""
    m = synth.tiny_model(5, P=20)
    off, idx = m.nbr_off.copy(), m.nbr_idx.copy()
    if case == "non_monotone":
        off[5], off[6] = off[6], off[5]
    elif case == "short_end":
        idx = idx[:-1].copy()  # offsets end beyond the neighbour array
    elif case == "self_neighbour":
        idx[off[3]] = 3
    else:
        idx[2] = -1
    with pytest.raises(rt.RtError) as ex:
        rt.Model.from_numpy(m.pos, off, idx)
    assert ex.value.code == -2


# ----------------------------------------------------------------------------- solve, FP64

def _solve_gpu(rt, m, model, ds, rays, org, n_o, precision, chi=None, eta=None, **kw):
    torch = _torch()
    dt = np.float64 if precision == rt.RT_F64 else np.float32
    chi = m.chi if chi is None else chi
    eta = m.eta if eta is None else eta
    return rt.solve(model, ds, rays, _t(chi.astype(dt)), _t(eta.astype(dt)), m.freq.len, m.freq.dx,
                    _t(m.I_bc, torch.float64), origins=org, n_origins=n_o, precision=precision, **kw)


@pytest.mark.parametrize("case", ["sphere", "tiny_moving", "tiny_2blocks", "tiny_F70", "lattice"])
def test_J_fp64(rt, orc, case):
    if case == "sphere":
        m, nside = synth.sphere_model(), 1
    elif case == "tiny_moving":
        m, nside = synth.tiny_model(6, P=60, F=8, moving=True), 2
    elif case == "tiny_2blocks":
        m, nside = synth.tiny_model(7, P=50, F=20, moving=True), 2
        m.freq = synth.FreqGrid(np.array([12, 8], np.int32), np.array([-3.0, -2.0]), np.array([0.5, 0.6]))
    elif case == "tiny_F70":
        m, nside = synth.tiny_model(8, P=40, F=70, moving=True), 1
    else:
        m, nside = synth.lattice_model(5, F=5), 1
        m.chi = np.random.default_rng(0).uniform(0.5, 2, m.chi.shape)
    model, ds, g, _, dirs, w2, org, oo = _trace_both(rt, orc, m, nside, None)
    J, u = _solve_gpu(rt, m, model, ds, g, org, m.P, rt.RT_F64, want_u=True)
    Je, ue = orc.compute_J(m, dirs, w2, origins=oo, want_u=True)
    assert _rel(u.cpu().numpy(), ue) <= TOL64
    assert _rel(J.cpu().numpy(), Je) <= TOL64


@pytest.fixture(scope="module")
def wind():
    return synth.wind_model()


@pytest.mark.parametrize("nside", [2, 4])
def test_J_wind_fp64_and_fp32(rt, orc, wind, nside):
    rng = np.random.default_rng(10 + nside)
    origins = rng.choice(wind.P, 400, replace=False)
    c32, e32, c64, e64 = synth.to_fp32_tables(wind.chi, wind.eta)
    model, ds, g, _, dirs, w2, org, oo = _trace_both(rt, orc, wind, nside, origins)
    Je = orc.compute_J(wind, dirs, w2, origins=oo, chi=c64, eta=e64)
    J64 = _solve_gpu(rt, wind, model, ds, g, org, len(oo), rt.RT_F64, chi=c64, eta=e64)
    assert _rel(J64.cpu().numpy(), Je) <= TOL64
    J32 = _solve_gpu(rt, wind, model, ds, g, org, len(oo), rt.RT_F32, chi=c32, eta=e32)
    err32 = _rel(J32.cpu().numpy().astype(np.float64), Je)
    assert err32 <= TOL32, err32


def test_fp32_error_on_optically_thin_and_thick_lines(rt, orc):
    # dtau spanning 1e-7 .. 1e3: with the rows carried per unit inner step every coefficient is its
    # FP64 value rounded once, which keeps the FP32 sweep within 1e-4 without an FP64 branch
    m = synth.tiny_model(9, P=60, F=16, moving=True)
    rng = np.random.default_rng(1)
    scale = 10.0 ** rng.uniform(-6, 3, (m.P, 1))
    m.chi = m.chi * scale
    m.eta = m.eta * scale
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    model, ds, g, _, dirs, w2, org, oo = _trace_both(rt, orc, m, 2, None)
    Je = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64)
    J32 = _solve_gpu(rt, m, model, ds, g, org, m.P, rt.RT_F32, chi=c32, eta=e32)
    assert _rel(J32.cpu().numpy().astype(np.float64), Je) <= TOL32


# ----------------------------------------------------------------------------- closed forms through the GPU

def test_sphere_centre_gpu(rt, orc):
    m = synth.sphere_model()
    model, ds, g, _, dirs, w2, org, oo = _trace_both(rt, orc, m, 1, np.array([0]))
    J = _solve_gpu(rt, m, model, ds, g, org, 1, rt.RT_F64).cpu().numpy()
    assert abs(J[0, 0] - (1 - np.exp(-2.0))) < 2e-2
    assert np.all(J[0] == J[0, 0])


@pytest.mark.parametrize("prec,tol", [(2, 1e-13), (1, 1e-5)])
def test_uniform_source_gives_J_equal_S(rt, orc, prec, tol):
    m = synth.tiny_model(11, P=60, F=12, moving=True)
    S0 = 0.625
    m.eta = m.chi * S0
    m.I_bc = np.full(m.F, S0)
    model, ds, g, _, dirs, w2, org, oo = _trace_both(rt, orc, m, 2, None)
    J = _solve_gpu(rt, m, model, ds, g, org, m.P, prec).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(J - S0)) <= tol


def test_galilean_invariance_gpu(rt, orc):
    m = synth.tiny_model(12, P=50, F=10)
    model, ds, g, _, dirs, w2, org, oo = _trace_both(rt, orc, m, 2, None)
    J0 = _solve_gpu(rt, m, model, ds, g, org, m.P, rt.RT_F64).cpu().numpy()
    m.vel = np.tile(np.array([[3.7, -1.2, 0.4]], np.float32), (m.P, 1))
    model_v = _gpu_model(rt, m)
    J1 = _solve_gpu(rt, m, model_v, ds, g, org, m.P, rt.RT_F64).cpu().numpy()
    assert np.array_equal(J0, J1)


# ----------------------------------------------------------------------------- schedules, plans, graphs

@pytest.mark.parametrize("prec", [1, 2])
def test_binned_schedule_bitwise_equal_direct(rt, orc, wind, prec):
    origins = np.arange(0, wind.P, 25)
    model, ds, g, _, dirs, w2, org, oo = _trace_both(rt, orc, wind, 2, origins)
    Jd = _solve_gpu(rt, wind, model, ds, g, org, len(oo), prec, schedule=rt.SCHED_DIRECT).cpu().numpy()
    for wpc, nb in ((0, 0), (4, 16), (64, 64)):
        Jb = _solve_gpu(rt, wind, model, ds, g, org, len(oo), prec, schedule=rt.SCHED_BINNED,
                        waves_per_cu=wpc, n_bins=nb).cpu().numpy()
        assert np.array_equal(Jd, Jb)


# walk 0: exact slots (default), 1: padded slots + compaction, 2: two passes
@pytest.mark.parametrize("schedule,walk,padded,lanes,group", [(0, 0, 0, 4, 8), (1, 1, 0, 8, 4), (1, 2, 0, 16, 8),
                                                             (2, 0, 0, 8, 4), (2, 1, -1, 4, 4), (2, 1, 0, 16, 8),
                                                             (2, 2, 0, 8, 8)])
def test_plan_graph_replays(rt, orc, wind, schedule, walk, padded, lanes, group):
    torch = _torch()
    origins = np.arange(0, wind.P, 50).astype(np.int32)
    model = _gpu_model(rt, wind)
    ds = rt.DirSet.uniform(2)
    c32, e32, c64, e64 = synth.to_fp32_tables(wind.chi, wind.eta)
    chi, eta = _t(c32), _t(e32)
    I_bc = _t(wind.I_bc, torch.float64)
    org = _t(origins)
    J = torch.empty((len(origins), wind.F), dtype=torch.float32, device="cuda")
    plan = rt.Plan(model, ds, chi, eta, wind.freq.len, wind.freq.dx, I_bc, J, origins=org,
                   precision=rt.RT_F32, schedule=schedule, padded_trace_budget=padded, trace_lanes=lanes,
                   group=group, walk=walk)
    ref = rt.compute_J_direct(model, ds, chi, eta, wind.freq.len, wind.freq.dx, I_bc, origins=org,
                       precision=rt.RT_F32).cpu().numpy()
    plan.run(use_graph=False)
    rt.sync_status()
    assert np.array_equal(J.cpu().numpy(), ref)
    for _ in range(3):
        J.zero_()
        plan.run(use_graph=True)
        rt.sync_status()
        assert np.array_equal(J.cpu().numpy(), ref)
        torch.cuda.synchronize()
    # the plan's lists are the oracle's
    off, ids, Z = plan.rays()
    _, dirs, _ = orc.dirset_uniform(2)
    e = orc.trace_all(wind, dirs, origins)
    _assert_rays_equal((off, ids, Z), e)
    prof = plan.profile(2)
    assert prof["sweep"] > 0 and prof["walk"] > 0
    rt.sync_status()


@pytest.fixture(scope="module")
def sph_cloud():
    return synth.sph_cloud_model(seed=402, P=12_000)


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_exact_walk_length_order_lists(rt, orc, sph_cloud, lanes):
    """The exact-slot walk takes each direction's rays in windows of 64 origins ordered by the
    lengths of the creation-time count: on an SPH-like cloud (rays from none to ~70 entries
    long, mean ~23), with 777 seeded origins (twelve full windows and a
    partial one), the plan's lists equal the oracle's walk bit for bit at every lane count,
    and J equals the same plan walked in two passes (which takes the origins in Morton order)."""
    torch = _torch()
    m = sph_cloud
    rng = np.random.default_rng(31)
    origins = np.sort(rng.choice(m.P, 777, replace=False)).astype(np.int32)
    model = _gpu_model(rt, m)
    ds = rt.DirSet.uniform(2)
    c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
    chi, eta = _t(c32), _t(e32)
    I_bc = _t(m.I_bc, torch.float64)
    org = _t(origins)
    Js = {}
    for walk in (rt.WALK_EXACT, rt.WALK_TWO_PASS):
        Js[walk] = torch.empty((len(origins), m.F), dtype=torch.float32, device="cuda")
        plan = rt.Plan(model, ds, chi, eta, m.freq.len, m.freq.dx, I_bc, Js[walk], origins=org,
                       precision=rt.RT_F32, schedule=rt.SCHED_SPATIAL, trace_lanes=lanes, walk=walk)
        plan.run(use_graph=True)
        rt.sync_status()
        if walk == rt.WALK_EXACT:
            _, dirs, _ = orc.dirset_uniform(2)
            e = orc.trace_all(m, dirs, origins)
            lens = np.diff(e[0])
            assert lens.min() == 0 and lens.max() > 2.5 * lens.mean()  # the lengths the order sorts differ widely
            _assert_rays_equal(plan.rays(), e)
        del plan
    assert np.array_equal(Js[rt.WALK_EXACT].cpu().numpy(), Js[rt.WALK_TWO_PASS].cpu().numpy())


def test_trace_write_flags_mismatched_offsets(rt, wind):
    """Writing at offsets that do not match the walk (here: every slot one entry too long)
    latches a capacity error instead of leaving the mismatch unnoticed."""
    torch = _torch()
    model = _gpu_model(rt, wind)
    ds = rt.DirSet.uniform(1)
    org = _t(np.arange(0, 200, dtype=np.int32))
    off, ids, Z = rt.trace(model, ds, origins=org)
    rt.sync_status()
    lens = torch.diff(off)
    off2 = torch.zeros_like(off)
    off2[1:] = torch.cumsum(lens + 1, 0)
    tot = int(off2[-1])
    ids2 = torch.empty(tot, dtype=torch.int32, device="cuda")
    Z2 = torch.empty(tot, dtype=torch.float64, device="cuda")
    rt.binding._check(rt.load().rt_trace_write(model._h, ds._h, org.data_ptr(), org.numel(), off2.data_ptr(),
                                               ids2.data_ptr(), Z2.data_ptr(), tot, rt.binding._stream(None)))
    with pytest.raises(rt.RtError) as ei:
        rt.sync_status()
    assert ei.value.code == -4
    rt.sync_status()


def test_empty_origin_list(rt):
    torch = _torch()
    m = synth.tiny_model(13, P=30, F=4)
    model = _gpu_model(rt, m)
    ds = rt.DirSet.uniform(1)
    org = torch.empty(0, dtype=torch.int32, device="cuda")
    off, ids, Z = rt.trace(model, ds, origins=org)
    assert off.numel() == 1 and int(off[0]) == 0 and ids.numel() == 0
    J = _solve_gpu(rt, m, model, ds, (off, ids, Z), org, 0, rt.RT_F64)
    assert J.shape == (0, m.F)


# ----------------------------------------------------------------------------- adaptive direction sets

@pytest.mark.parametrize("lmin,lmax", [(1, 4), (0, 3), (2, 3)])
def test_adaptive_sets_bitwise(rt, orc, wind, lmin, lmax):
    torch = _torch()
    rng = np.random.default_rng(lmin * 10 + lmax)
    sample = rng.choice(wind.P, 10_000, replace=False).astype(np.int32)
    origins = rng.choice(wind.P, 300, replace=False).astype(np.int32)
    model = _gpu_model(rt, wind)
    ds = rt.DirSet.adaptive(model, lmin, lmax, _t(sample), origins=_t(origins))
    pix, lev, dirs, w2 = ds.export()
    e_pix, e_lev, e_dirs, e_w2 = orc.dirset_adaptive(wind, lmin, lmax, sample, origins=origins)
    assert np.array_equal(lev, e_lev)
    assert np.array_equal(pix, e_pix)
    assert np.array_equal(dirs.view(np.uint64), e_dirs.view(np.uint64))
    assert np.array_equal(w2, e_w2)
    assert ds.info()["R"] == orc.dirset_adaptive_R(lmin, lmax)
    del torch


def test_adaptive_J_and_lmax_identity(rt, orc, wind):
    torch = _torch()
    rng = np.random.default_rng(77)
    sample = rng.choice(wind.P, 10_000, replace=False).astype(np.int32)
    origins = rng.choice(wind.P, 120, replace=False).astype(np.int32)
    model = _gpu_model(rt, wind)
    org = _t(origins)
    ds = rt.DirSet.adaptive(model, 1, 3, _t(sample), origins=org)
    pix, lev, dirs, w2 = ds.export()
    rays = rt.trace(model, ds, origins=org)
    e = orc.trace_all(wind, dirs, origins)
    _assert_rays_equal(rays, e)
    c32, e32, c64, e64 = synth.to_fp32_tables(wind.chi, wind.eta)
    J64, u64 = _solve_gpu(rt, wind, model, ds, rays, org, len(origins), rt.RT_F64, chi=c64, eta=e64, want_u=True)
    Je = orc.compute_J(wind, dirs, w2, origins=origins, chi=c64, eta=e64)
    assert _rel(J64.cpu().numpy(), Je) <= TOL64
    # Section 3.2.1: the maximally refined directions are the dense regular ones, with the same u
    du = rt.DirSet.uniform(8)
    upix = du.export()[0]
    where = {int(p): i for i, p in enumerate(upix)}
    rays_u = rt.trace(model, du, origins=org)
    J_u, u_u = _solve_gpu(rt, wind, model, du, rays_u, org, len(origins), rt.RT_F64, chi=c64, eta=e64, want_u=True)
    u64, u_u = u64.cpu().numpy(), u_u.cpu().numpy()
    n = 0
    for o in range(len(origins)):
        for r in np.nonzero(lev[o] == 3)[0]:
            assert u64[o, r].tobytes() == u_u[o, where[int(pix[o, r])]].tobytes()
            n += 1
    assert n == len(origins) * 96
    del torch


# ----------------------------------------------------------------------------- batching, octree, autotuner

def test_octree_cloud_parity(rt, orc):
    # touching-leaf adjacency: many exact distance ties, two frequency blocks
    m = synth.octree_model(seed=31, lmin=3, lmax=5, target=3000)
    rng = np.random.default_rng(8)
    origins = rng.choice(m.P, 200, replace=False)
    model, ds, g, e, dirs, w2, org, oo = _trace_both(rt, orc, m, 2, origins)
    _assert_rays_equal(g, e)
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    Je = orc.compute_J(m, dirs, w2, origins=oo, chi=c64, eta=e64)
    J64 = _solve_gpu(rt, m, model, ds, g, org, len(oo), rt.RT_F64, chi=c64, eta=e64)
    assert _rel(J64.cpu().numpy(), Je) <= TOL64
    J32 = _solve_gpu(rt, m, model, ds, g, org, len(oo), rt.RT_F32, chi=c32, eta=e32)
    assert _rel(J32.cpu().numpy().astype(np.float64), Je) <= TOL32


def test_packed_half_waves_match_unpacked(rt):
    """65..96 frequencies: the second 64-frequency chunks of two pairs share one wave, 32 lanes
    each.  The octree cloud (F = 96, blocks 48 + 48) against the same cloud cut to its
    frequencies 32..95 (blocks 16 + 48, F = 64, nothing packed): u of the second block, and so
    J there, is the same bit for bit, in FP32 and FP64, eagerly and with the persistent launch."""
    torch = _torch()
    m = synth.octree_model(seed=31, lmin=3, lmax=5, target=3000)
    assert m.F == 96 and list(m.freq.len) == [48, 48]
    model = _gpu_model(rt, m)
    ds = rt.DirSet.uniform(2)
    rng = np.random.default_rng(12)
    org = _t(np.sort(rng.choice(m.P, 300, replace=False)).astype(np.int32))
    rays = rt.trace(model, ds, origins=org)
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    dx = list(m.freq.dx)
    for prec, chi, eta in ((rt.RT_F32, c32, e32), (rt.RT_F64, c64, e64)):
        for schedule in (rt.SCHED_DIRECT, rt.SCHED_BINNED):
            JA, uA = rt.solve(model, ds, rays, _t(chi), _t(eta), [48, 48], dx, _t(m.I_bc, torch.float64),
                              origins=org, precision=prec, want_u=True, schedule=schedule)
            JB, uB = rt.solve(model, ds, rays, _t(chi[:, 32:]), _t(eta[:, 32:]), [16, 48], dx,
                              _t(m.I_bc[32:], torch.float64), origins=org, precision=prec, want_u=True,
                              schedule=schedule)
            rt.sync_status()
            a, b = uA.cpu().numpy(), uB.cpu().numpy()
            assert np.array_equal(a[:, :, 48:], b[:, :, 16:])
            assert np.array_equal(JA.cpu().numpy()[:, 48:], JB.cpu().numpy()[:, 16:])


@pytest.mark.parametrize("lmin,lmax", [(1, 3), (0, 3)])
def test_adaptive_sets_with_96_frequencies(rt, orc, lmin, lmax):
    """Per-origin direction sets on the 96-frequency octree cloud: with an even pair count (132)
    the packed half waves take each pair's own direction from the origin's set, with an odd one
    (69) nothing is packed; FP64 and FP32 against the oracle."""
    torch = _torch()
    m = synth.octree_model(seed=31, lmin=3, lmax=5, target=3000)
    rng = np.random.default_rng(lmin + 13)
    sample = rng.choice(m.P, 2000, replace=False).astype(np.int32)
    origins = rng.choice(m.P, 80, replace=False).astype(np.int32)
    model = _gpu_model(rt, m)
    org = _t(origins)
    ds = rt.DirSet.adaptive(model, lmin, lmax, _t(sample), origins=org)
    assert ds.info()["R"] == orc.dirset_adaptive_R(lmin, lmax)
    _, _, dirs, w2 = ds.export()
    rays = rt.trace(model, ds, origins=org)
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    Je = orc.compute_J(m, dirs, w2, origins=origins, chi=c64, eta=e64)
    J64 = _solve_gpu(rt, m, model, ds, rays, org, len(origins), rt.RT_F64, chi=c64, eta=e64)
    assert _rel(J64.cpu().numpy(), Je) <= TOL64
    J32 = _solve_gpu(rt, m, model, ds, rays, org, len(origins), rt.RT_F32, chi=c32, eta=e32)
    assert _rel(J32.cpu().numpy().astype(np.float64), Je) <= TOL32
    del torch


def test_batched_union(rt, orc):
    torch = _torch()
    ms = synth.sph_batch_models(n_models=5, lo=800, hi=3000, seed0=900)
    u = synth.concat_models(ms)
    model = _gpu_model(rt, u)
    ds = rt.DirSet.uniform(2)
    c32, e32, c64, e64 = synth.to_fp32_tables(u.chi, u.eta)
    J = torch.empty((u.P, u.F), dtype=torch.float32, device="cuda")
    plan = rt.Plan(model, ds, _t(c32), _t(e32), u.freq.len, u.freq.dx, _t(u.I_bc, torch.float64), J,
                   n_origins=u.P, precision=rt.RT_F32, schedule=rt.SCHED_BINNED)
    plan.run()
    rt.sync_status()
    off, ids, Z = (x.cpu().numpy() for x in plan.rays())
    # no ray leaves its own model
    starts = u.meta["offsets"]
    owner = np.searchsorted(starts, np.arange(u.P), side="right") - 1
    ray_origin = np.repeat(np.arange(u.P), 2 * ds.R)
    ray_of_entry = np.repeat(np.arange(len(off) - 1), np.diff(off))
    assert np.array_equal(owner[ids], owner[ray_origin[ray_of_entry]])
    # sampled origins of every model against the oracle on the union
    rng = np.random.default_rng(9)
    origins = np.concatenate([rng.choice(np.arange(starts[k], starts[k + 1]), 20, replace=False)
                              for k in range(len(ms))]).astype(np.int32)
    _, dirs, w2 = orc.dirset_uniform(2)
    Je = orc.compute_J(u, dirs, w2, origins=origins, chi=c64, eta=e64)
    assert _rel(J.cpu().numpy()[origins].astype(np.float64), Je) <= TOL32


def test_autotune_and_cache(rt, wind, tmp_path):
    torch = _torch()
    origins = np.arange(0, wind.P, 20).astype(np.int32)
    model = _gpu_model(rt, wind)
    ds = rt.DirSet.uniform(2)
    c32, e32, _, _ = synth.to_fp32_tables(wind.chi, wind.eta)
    chi, eta = _t(c32), _t(e32)
    I_bc = _t(wind.I_bc, torch.float64)
    J = torch.empty((len(origins), wind.F), dtype=torch.float32, device="cuda")
    cache = str(tmp_path / "tune.txt")
    opts, ms = rt.autotune(model, ds, chi, eta, wind.freq.len, wind.freq.dx, I_bc, J, origins=_t(origins),
                           n_runs=1, cache_path=cache)
    assert opts["schedule"] in (0, 1, 2) and opts["group"] in (4, 8) and opts["trace_lanes"] in (4, 8, 16)
    assert ms > 0 and open(cache).read().count("\n") == 1
    opts2, ms2 = rt.autotune(model, ds, chi, eta, wind.freq.len, wind.freq.dx, I_bc, J, origins=_t(origins),
                             n_runs=1, cache_path=cache)
    assert opts2 == opts and abs(ms2 - ms) < 1e-3 and open(cache).read().count("\n") == 1
    plan = rt.Plan(model, ds, chi, eta, wind.freq.len, wind.freq.dx, I_bc, J, origins=_t(origins), **opts)
    plan.run()
    rt.sync_status()
    ref = rt.compute_J_direct(model, ds, chi, eta, wind.freq.len, wind.freq.dx, I_bc, origins=_t(origins))
    assert np.array_equal(J.cpu().numpy(), ref.cpu().numpy())
    # re-captured with every schedule and tile option: the same result, bit for bit
    for sc, g, la, wpc in ((2, 8, 16, 0), (1, 4, 4, 16), (0, 8, 8, 0), (2, 4, 8, 0)):
        J.zero_()
        plan.retune(schedule=sc, group=g, trace_lanes=la, waves_per_cu=wpc, n_bins=64 if sc == 1 else 0)
        plan.run()
        rt.sync_status()
        assert np.array_equal(J.cpu().numpy(), ref.cpu().numpy())


@pytest.mark.parametrize("blocks", ["one", "two_same_dx", "two_dx", "static"])
@pytest.mark.parametrize("fp64", [False, True])
def test_plan_moving_blocks_bitwise(rt, blocks, fp64):
    """Plans (spatial schedule, graph replays) give the direct solve's bits for
    one block, two blocks of one width, two blocks of different widths and a
    static model, and still do after the tables change in place between runs."""
    torch = _torch()
    m = synth.tiny_model(81, P=150, F=20, moving=blocks != "static")
    if blocks == "two_same_dx":
        m.freq = synth.FreqGrid(np.array([12, 8], np.int32), np.array([-3.0, -2.0]), np.array([0.5, 0.5]))
    elif blocks == "two_dx":
        m.freq = synth.FreqGrid(np.array([12, 8], np.int32), np.array([-3.0, -2.0]), np.array([0.5, 0.7]))
    prec = rt.RT_F64 if fp64 else rt.RT_F32
    dt = np.float64 if fp64 else np.float32
    model = _gpu_model(rt, m)
    ds = rt.DirSet.uniform(2)
    chi, eta = _t(m.chi.astype(dt)), _t(m.eta.astype(dt))
    I_bc = _t(m.I_bc, torch.float64)
    J = torch.empty((m.P, m.F), dtype=chi.dtype, device="cuda")
    plan = rt.Plan(model, ds, chi, eta, m.freq.len, m.freq.dx, I_bc, J, n_origins=m.P, precision=prec,
                   schedule=rt.SCHED_SPATIAL)
    for scale in (1.0, 3.0):
        chi.mul_(scale)
        ref = rt.compute_J_direct(model, ds, chi, eta, m.freq.len, m.freq.dx, I_bc, precision=prec).cpu().numpy()
        for use_graph in (False, True, True):
            J.zero_()
            plan.run(use_graph=use_graph)
            rt.sync_status()
            assert np.array_equal(J.cpu().numpy(), ref)


def test_plan_buffer_cache(rt, wind):
    """Destroyed plans leave their large buffers in the library's cache; the next
    plans take them (no new allocation) and give the same bits as fresh ones, and
    releasing the cache empties it."""
    import gc
    torch = _torch()
    model = _gpu_model(rt, wind)
    ds = rt.DirSet.uniform(2)
    c32, e32, _, _ = synth.to_fp32_tables(wind.chi, wind.eta)
    chi, eta = _t(c32), _t(e32)
    I_bc = _t(wind.I_bc, torch.float64)
    rt.release_cached_memory()
    assert rt.cached_memory() == 0
    n = 20_000
    org = _t(np.arange(n, dtype=np.int32))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]

    def run(origins, k):
        J = torch.empty((k, wind.F), dtype=torch.float32, device="cuda")
        plan = rt.Plan(model, ds, chi, eta, wind.freq.len, wind.freq.dx, I_bc, J, origins=origins,
                       precision=rt.RT_F32, schedule=rt.SCHED_SPATIAL)
        plan.run()
        rt.sync_status()
        out = J.cpu().numpy()
        del plan
        gc.collect()
        return out

    ref = run(org, n)
    held = rt.cached_memory()
    assert held >= 3 * (64 << 20)  # ids, Z and u of the plan
    again = run(org, n)
    assert np.array_equal(again, ref)
    assert rt.cached_memory() == held  # the second plan took the same buffers and returned them
    half = run(org[: n // 2], n // 2)  # smaller plans fit the cached blocks too
    direct = rt.compute_J_direct(model, ds, chi, eta, wind.freq.len, wind.freq.dx, I_bc, origins=org[: n // 2],
                          precision=rt.RT_F32).cpu().numpy()
    assert np.array_equal(half, direct)
    rt.release_cached_memory()
    assert rt.cached_memory() == 0
    assert rt.plan_memory() == 0  # no plan is alive
    # every plan buffer went back to the device
    del direct
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"device memory free before {free0 / 2**30:.3f} GiB, after {free1 / 2**30:.3f} GiB", flush=True)
    assert free1 >= free0 - (64 << 20)


def test_full_size_plan_sampled_parity(rt, orc, wind):
    """The headline configuration as the benchmark times it: one plan over all 50 000
    wind origins at nside 4, FP32 sweep, library defaults (spatial schedule, load
    group 4, 4 lanes per ray, exact-slot walk), replayed as a graph.  Sampled origins
    (the oracle walks and solves them one by one): their ray lists bit-exact, their
    J within 1e-4 of the FP64 oracle on the same FP32 tables."""
    torch = _torch()
    nside = 4
    model = _gpu_model(rt, wind)
    ds = rt.DirSet.uniform(nside)
    _, dirs, w2 = orc.dirset_uniform(nside)
    c32, e32, c64, e64 = synth.to_fp32_tables(wind.chi, wind.eta)
    J = torch.empty((wind.P, wind.F), dtype=torch.float32, device="cuda")
    plan = rt.Plan(model, ds, _t(c32), _t(e32), wind.freq.len, wind.freq.dx, _t(wind.I_bc, torch.float64), J,
                   n_origins=wind.P, precision=rt.RT_F32, schedule=rt.SCHED_SPATIAL)
    for _ in range(2):
        plan.run(use_graph=True)
    rt.sync_status()
    rng = np.random.default_rng(77)
    sample = np.sort(rng.choice(wind.P, 300, replace=False)).astype(np.int32)
    sample[0], sample[-1] = 0, wind.P - 1  # the first and last slots of the lists too
    # the sampled origins' ray lists: each origin's 2R rays are one contiguous run
    off, ids, Z = plan.rays()
    two_r = 2 * ds.R
    off_h = off.cpu().numpy()
    idx = torch.as_tensor(np.concatenate([np.arange(off_h[o * two_r], off_h[(o + 1) * two_r]) for o in sample]),
                          device="cuda")
    g_ids, g_Z = ids[idx].cpu().numpy(), Z[idx].cpu().numpy()
    g_off = np.concatenate([[0], np.cumsum(np.concatenate([np.diff(off_h[o * two_r:(o + 1) * two_r + 1])
                                                           for o in sample]))])
    e_off, e_ids, e_Z = orc.trace_all(wind, dirs, sample)
    assert np.array_equal(g_off, e_off)
    assert np.array_equal(g_ids, e_ids)
    assert np.array_equal(g_Z.view(np.uint64), e_Z.view(np.uint64))
    Je = orc.compute_J(wind, dirs, w2, origins=sample, chi=c64, eta=e64)
    err = _rel(J[_t(sample).long()].cpu().numpy().astype(np.float64), Je)
    print(f"full-size plan: {plan.info()['total']} entries, sampled J max rel {err:.2e}", flush=True)
    assert err <= TOL32


@pytest.mark.parametrize("n_org", [1, 3, 7, 33])
def test_persistent_queue_small_and_ragged(rt, orc, n_org):
    """The persistent launch takes 16 items per queue atomic: item counts below one
    chunk, and counts that leave a partial last chunk (nside 1: 6 pairs per origin,
    two 64-frequency chunks at F = 70), give the direct launch's bits, eagerly and
    from a binned plan replayed twice; FP64 also against the oracle."""
    torch = _torch()
    m = synth.tiny_model(90 + n_org, P=40, F=70, moving=True)
    origins = np.arange(n_org, dtype=np.int32) * 3 % m.P
    model, ds, g, _, dirs, w2, org, oo = _trace_both(rt, orc, m, 1, origins)
    Jd = _solve_gpu(rt, m, model, ds, g, org, len(oo), rt.RT_F64, schedule=rt.SCHED_DIRECT).cpu().numpy()
    assert _rel(Jd, orc.compute_J(m, dirs, w2, origins=oo)) <= TOL64
    Jb = _solve_gpu(rt, m, model, ds, g, org, len(oo), rt.RT_F64, schedule=rt.SCHED_BINNED).cpu().numpy()
    assert np.array_equal(Jd, Jb)
    J = torch.empty((len(oo), m.F), dtype=torch.float64, device="cuda")
    plan = rt.Plan(model, ds, _t(m.chi), _t(m.eta), m.freq.len, m.freq.dx, _t(m.I_bc, torch.float64), J,
                   origins=org, precision=rt.RT_F64, schedule=rt.SCHED_BINNED, waves_per_cu=1)
    for _ in range(2):
        J.zero_()
        plan.run(use_graph=True)
        rt.sync_status()
        assert np.array_equal(J.cpu().numpy(), Jd)
