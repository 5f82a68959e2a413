"""GPU parity of the whole-path entry points: rt_compute_J (chunked inside a caller
workspace), rt_batch / rt_compute_J_batched (many models as one disjoint union) and
rt_closure_J (the learned closure in one call).

Each is compared bit for bit with the low-level calls (rt_trace_count, rt_trace_write,
rt_solve; the closure's steps one by one), which the other GPU tests pin to the oracle,
and on the FP64 path also with the oracle itself (1e-12)."""
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


def _gpu_model(rt, m):
    return rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def _bar_model(n=240, w=3, F=16, seed=5):
    """A long thin lattice (n x w x w, face neighbours, slightly jittered): rays with an x
    component run the length of the bar, so rays average far more entries than 64."""
    rng = np.random.default_rng(seed)
    g = np.stack(np.meshgrid(np.arange(n), np.arange(w), np.arange(w), indexing="ij"), -1).reshape(-1, 3)
    pos = g.astype(np.float64) + rng.uniform(-0.05, 0.05, g.shape)
    lin = lambda i, j, k: (i * w + j) * w + k  # noqa: E731
    a, b = [], []
    for i in range(n):
        for j in range(w):
            for k in range(w):
                if i + 1 < n:
                    a.append(lin(i, j, k)); b.append(lin(i + 1, j, k))  # noqa: E702
                if j + 1 < w:
                    a.append(lin(i, j, k)); b.append(lin(i, j + 1, k))  # noqa: E702
                if k + 1 < w:
                    a.append(lin(i, j, k)); b.append(lin(i, j, k + 1))  # noqa: E702
    off, idx = synth.csr_from_edges(len(pos), np.array(a), np.array(b))
    P = len(pos)
    freq = synth.FreqGrid.uniform(1, F)
    chi = rng.uniform(0.05, 0.4, (P, F))
    eta = chi * rng.uniform(0.2, 1.5, (P, F))
    vel = rng.normal(0.0, 0.8, (P, 3)).astype(np.float32)
    return synth.Model("bar", pos, off, idx, vel, chi, eta, freq, rng.uniform(0.0, 0.3, F), meta={})


@pytest.fixture(scope="module")
def wind():
    return synth.wind_model(seed=2, P=20_000)


@pytest.mark.parametrize("schedule", ["spatial", "binned", "direct"])
def test_compute_J_chunked_equals_direct(rt, wind, schedule):
    """Shuffled origin list, a workspace of about 1/25 of what one chunk needs: many chunks
    in Morton order, J and u scattered back to list order, bit for bit the direct solve."""
    torch = _torch()
    sc = {"spatial": rt.SCHED_SPATIAL, "binned": rt.SCHED_BINNED, "direct": rt.SCHED_DIRECT}[schedule]
    model = _gpu_model(rt, wind)
    ds = rt.DirSet.uniform(2)
    c32, e32, _, _ = synth.to_fp32_tables(wind.chi, wind.eta)
    chi, eta, I_bc = _t(c32), _t(e32), _t(wind.I_bc, torch.float64)
    rng = np.random.default_rng(4)
    org = _t(rng.permutation(wind.P)[:6000].astype(np.int32))
    ref, uref = rt.solve(model, ds, rt.trace(model, ds, origins=org), chi, eta, wind.freq.len, wind.freq.dx, I_bc,
                         origins=org, want_u=True)
    full = rt.compute_J_workspace(ds, 6000, wind.F, schedule=sc)
    J, u = rt.compute_J(model, ds, chi, eta, wind.freq.len, wind.freq.dx, I_bc, origins=org, schedule=sc,
                        ws_bytes=full // 25, want_u=True)
    rt.sync_status()
    assert np.array_equal(J.cpu().numpy(), ref.cpu().numpy())
    assert np.array_equal(u.cpu().numpy(), uref.cpu().numpy())
    # every origin (NULL list), one chunk
    Jall = rt.compute_J(model, ds, chi, eta, wind.freq.len, wind.freq.dx, I_bc, schedule=sc)
    rt.sync_status()
    sub = org.long()
    assert np.array_equal(Jall[sub].cpu().numpy(), ref.cpu().numpy())


def test_compute_J_long_rays_window_cut(rt, orc):
    """Rays averaging well over the 64 entries the window is sized for, in a workspace far below
    one chunk: each chunk is the longest prefix of the counted window whose lists fit, and the
    rest of the window keeps its counts for the next chunks.  FP64 against the oracle, FP32
    against the direct solve bit for bit."""
    torch = _torch()
    m = _bar_model()
    model = _gpu_model(rt, m)
    ds = rt.DirSet.uniform(1)
    _, dirs, w2 = orc.dirset_uniform(1)
    I_bc = _t(m.I_bc, torch.float64)
    off, _, _ = rt.trace(model, ds)
    mean = float(off[-1].item()) / (m.P * 2 * ds.R)
    assert mean > 70, mean
    ws = rt.compute_J_workspace(ds, m.P, m.F, precision=rt.RT_F64, mean_entries=mean) // 12
    J = rt.compute_J(model, ds, _t(m.chi), _t(m.eta), m.freq.len, m.freq.dx, I_bc, precision=rt.RT_F64,
                     ws_bytes=ws)
    rt.sync_status()
    rng = np.random.default_rng(2)
    sample = np.sort(rng.choice(m.P, 150, replace=False)).astype(np.int32)
    Je = orc.compute_J(m, dirs, w2, origins=sample)
    assert _rel(J.cpu().numpy()[sample], Je) <= TOL64
    c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
    J32 = rt.compute_J(model, ds, _t(c32), _t(e32), m.freq.len, m.freq.dx, I_bc, ws_bytes=ws)
    ref = rt.compute_J_direct(model, ds, _t(c32), _t(e32), m.freq.len, m.freq.dx, I_bc)
    rt.sync_status()
    assert np.array_equal(J32.cpu().numpy(), ref.cpu().numpy())


def test_compute_J_adaptive_set(rt, orc):
    """Per-origin (adaptive) direction sets keep the list order and offset their tables per
    chunk; FP64 against the oracle with the same sets."""
    torch = _torch()
    m = synth.tiny_model(71, P=300, F=10, moving=True)
    model = _gpu_model(rt, m)
    rng = np.random.default_rng(3)
    origins = rng.permutation(m.P)[:120].astype(np.int32)
    sample = rng.choice(m.P, 200, replace=False).astype(np.int32)
    ds = rt.DirSet.adaptive(model, 0, 2, _t(sample), origins=_t(origins))
    _, _, dirs, w2 = ds.export()
    ws = rt.compute_J_workspace(ds, len(origins), m.F, precision=rt.RT_F64) // 8
    J = rt.compute_J(model, ds, _t(m.chi), _t(m.eta), m.freq.len, m.freq.dx, _t(m.I_bc, torch.float64),
                     origins=_t(origins), precision=rt.RT_F64, ws_bytes=ws)
    rt.sync_status()
    Je = orc.compute_J(m, dirs, w2, origins=origins)
    assert _rel(J.cpu().numpy(), Je) <= TOL64


def test_trace_in_one_call(rt, wind):
    """rt_trace (count, scan, write in one call) gives the two-call lists bit for bit; with too
    little capacity it still reports the total, truncates, and latches RT_ERR_CAPACITY."""
    torch = _torch()
    model = _gpu_model(rt, wind)
    ds = rt.DirSet.uniform(2)
    org = _t(np.arange(0, wind.P, 7).astype(np.int32))
    off, ids, Z = rt.trace(model, ds, origins=org)
    total = int(off[-1].item())
    off1, ids1, Z1, t1 = rt.trace_once(model, ds, total, origins=org)
    rt.sync_status()
    assert t1 == total
    assert torch.equal(off1, off) and torch.equal(ids1[:total], ids) and torch.equal(Z1[:total], Z)
    _, ids2, _, t2 = rt.trace_once(model, ds, total // 2, origins=org)
    assert t2 == total
    with pytest.raises(rt.RtError) as e:
        rt.sync_status()
    assert e.value.code == -4
    rt.sync_status()  # cleared


def test_compute_J_workspace_too_small(rt, wind):
    torch = _torch()
    model = _gpu_model(rt, wind)
    ds = rt.DirSet.uniform(2)
    c32, e32, _, _ = synth.to_fp32_tables(wind.chi, wind.eta)
    with pytest.raises(rt.RtError) as e:
        rt.compute_J(model, ds, _t(c32), _t(e32), wind.freq.len, wind.freq.dx, _t(wind.I_bc, torch.float64),
                     ws_bytes=4096)
    assert e.value.code == -4


def _batch_models():
    ms = synth.sph_batch_models(n_models=4, lo=800, hi=3000, seed0=920)
    st = synth.tiny_model(33, P=500, F=64, moving=False)  # a static model among moving ones
    st.freq = ms[0].freq
    st.I_bc = ms[0].I_bc.copy()  # one grid and one boundary intensity for the whole batch
    return ms + [st]


def _rays_np(views, n_rays):
    off, ids, Z = views
    off = off[:n_rays + 1].cpu().numpy()
    return off, ids[:int(off[-1])].cpu().numpy(), Z[:int(off[-1])].cpu().numpy()


def test_batch_union_order(rt):
    """The union renumbers each model's points into the Morton order of its positions: the
    union index is a permutation inside each model's id range, consecutive union ids are
    close in space, and every ray list of the union is the model's own list with its ids
    renamed, bit for bit (lengths, ids, Z) -- also on a lattice, whose rays meet exact
    distance ties that the walk breaks by the model's own id order."""
    torch = _torch()
    ms = _batch_models()[:2]
    lat = synth.lattice_model(6, F=ms[0].F)
    lat.freq, lat.I_bc = ms[0].freq, ms[0].I_bc.copy()
    ms.append(lat)
    models = [_gpu_model(rt, m) for m in ms]
    ds = rt.DirSet.uniform(2)
    two_r = 2 * ds.R
    chis, etas = [], []
    for m in ms:
        c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
        chis.append(_t(c32))
        etas.append(_t(e32))
    I_bc = _t(ms[0].I_bc, torch.float64)
    Js = [torch.empty((m.P, m.F), dtype=torch.float32, device="cuda") for m in ms]
    b = rt.Batch(models, ds, chis, etas, ms[0].freq.len, ms[0].freq.dx, I_bc, Js, schedule=rt.SCHED_SPATIAL)
    b.run()
    rt.sync_status()
    uidx = b.union_index().cpu().numpy().astype(np.int64)
    base = np.concatenate([[0], np.cumsum([m.P for m in ms])])
    P_tot = int(base[-1])
    off_u, ids_u, Z_u = _rays_np(b.rays_view(), P_tot * two_r)
    for k, (m, mo) in enumerate(zip(ms, models)):
        seg = uidx[base[k]:base[k + 1]]
        assert np.array_equal(np.sort(seg), np.arange(base[k], base[k + 1]))
        if m.name == "sph":  # consecutive union ids are neighbours in space, not in generation order
            inv = np.empty(m.P, np.int64)
            inv[seg - base[k]] = np.arange(m.P)
            step_u = np.linalg.norm(np.diff(m.pos[inv], axis=0), axis=1).mean()
            step_m = np.linalg.norm(np.diff(m.pos, axis=0), axis=1).mean()
            assert step_u < 0.5 * step_m
        J = torch.empty((m.P, m.F), dtype=torch.float32, device="cuda")
        plan = rt.Plan(mo, ds, chis[k], etas[k], m.freq.len, m.freq.dx, I_bc, J, n_origins=m.P,
                       precision=rt.RT_F32, schedule=rt.SCHED_SPATIAL)
        plan.run()
        rt.sync_status()
        off_a, ids_a, Z_a = _rays_np(plan.rays_view(), m.P * two_r)
        len_a = np.diff(off_a)
        ray_u = (seg[np.arange(m.P)][:, None] * two_r + np.arange(two_r)[None, :]).ravel()
        assert np.array_equal(np.diff(off_u)[ray_u], len_a)
        src = np.repeat(off_u[ray_u], len_a) + (np.arange(len(ids_a)) - np.repeat(off_a[:-1], len_a))
        assert np.array_equal(ids_u[src], uidx[base[k] + ids_a])
        assert np.array_equal(Z_u[src].view(np.uint64), Z_a.view(np.uint64))
        assert np.array_equal(Js[k].cpu().numpy(), J.cpu().numpy())
        del plan


@pytest.mark.parametrize("schedule", ["binned", "spatial"])
def test_batch_equals_each_model_alone(rt, schedule):
    """The union's J of every model equals that model solved alone, bit for bit (positions
    are not moved, each model's points are renumbered into Morton order on the device and
    its neighbour rows keep the model's own id order), across graph replays, after the
    tables change in place, with one table of row stride > F, and after re-tuning."""
    torch = _torch()
    sc = rt.SCHED_BINNED if schedule == "binned" else rt.SCHED_SPATIAL
    ms = _batch_models()
    models = [_gpu_model(rt, m) for m in ms]
    ds = rt.DirSet.uniform(2)
    chis, etas = [], []
    for k, m in enumerate(ms):
        c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
        if k == 1:  # row stride 70 > F
            c32 = np.pad(c32, ((0, 0), (0, 6)), constant_values=1.0)
            e32 = np.pad(e32, ((0, 0), (0, 6)), constant_values=1.0)
        chis.append(_t(c32))
        etas.append(_t(e32))
    F = ms[0].F
    I_bc = _t(ms[0].I_bc, torch.float64)
    Js = [torch.empty((m.P, F), dtype=torch.float32, device="cuda") for m in ms]
    b = rt.Batch(models, ds, chis, etas, ms[0].freq.len, ms[0].freq.dx, I_bc, Js, schedule=sc)
    assert b.union() == (sum(m.P for m in ms), sum(m.E for m in ms))
    # the inner plan runs on the union's tables before any batch replay (the autotuner does this):
    # they hold the models' values from creation on, so nothing non-finite is latched
    b.profile(1)
    rt.sync_status()

    def refs():
        return [rt.compute_J_direct(mo, ds, c[:, :F].contiguous(), e[:, :F].contiguous(), m.freq.len, m.freq.dx,
                                    I_bc).cpu().numpy() for mo, c, e, m in zip(models, chis, etas, ms)]

    ref = refs()
    for use_graph in (False, True, True):
        for J in Js:
            J.zero_()
        b.run(use_graph=use_graph)
        rt.sync_status()
        for J, r in zip(Js, ref):
            assert np.array_equal(J.cpu().numpy(), r)
    chis[2].mul_(1.7)
    ref = refs()
    b.run()
    rt.sync_status()
    for J, r in zip(Js, ref):
        assert np.array_equal(J.cpu().numpy(), r)
    opts, ms_step = b.autotune(n_runs=1)
    assert ms_step > 0 and opts["schedule"] in (0, 1, 2)
    for J in Js:
        J.zero_()
    b.run()
    rt.sync_status()
    for J, r in zip(Js, ref):
        assert np.array_equal(J.cpu().numpy(), r)
    # the one-shot call
    Jo = rt.compute_J_batched(models, ds, chis, etas, ms[0].freq.len, ms[0].freq.dx, I_bc, schedule=sc)
    for J, r in zip(Jo, ref):
        assert np.array_equal(J.cpu().numpy(), r)


def test_batch_fp64_against_oracle(rt, orc):
    torch = _torch()
    ms = _batch_models()
    models = [_gpu_model(rt, m) for m in ms]
    ds = rt.DirSet.uniform(2)
    _, dirs, w2 = orc.dirset_uniform(2)
    Js = rt.compute_J_batched(models, ds, [_t(m.chi) for m in ms], [_t(m.eta) for m in ms], ms[0].freq.len,
                              ms[0].freq.dx, _t(ms[0].I_bc, torch.float64), precision=rt.RT_F64)
    rng = np.random.default_rng(12)
    for m, J in zip(ms, Js):
        sample = np.sort(rng.choice(m.P, 25, replace=False)).astype(np.int32)
        assert _rel(J.cpu().numpy()[sample], orc.compute_J(m, dirs, w2, origins=sample)) <= TOL64


def test_closure_J_equals_its_steps(rt):
    """rt_closure_J against the closure's steps called one by one (coarse solve, features,
    standardisation, network, flags, fine solve of the flagged points, merge): the same J
    bit for bit and the same flagged set, with no fallback, every point falling back (then
    J is the plain fine solve) and a bound between."""
    torch = _torch()
    m = synth.wind_model(seed=14, P=3000)
    model = _gpu_model(rt, m)
    c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
    chi, eta, I_bc = _t(c32), _t(e32), _t(m.I_bc, torch.float64)
    d1, d8 = rt.DirSet.uniform(1), rt.DirSet.uniform(4)
    J1, u1 = rt.solve(model, d1, rt.trace(model, d1), chi, eta, m.freq.len, m.freq.dx, I_bc, want_u=True)
    x = _t(m.freq.x().astype(np.float32))
    feat = rt.closure_features(model, chi, eta, x, J1, u=u1)
    sums = rt.closure_feature_stats(feat).cpu().numpy()
    n = feat.shape[0]
    mean = sums[:16] / n
    var = np.maximum(sums[16:] / n - mean * mean, 0.0)
    inv = np.where(var > 1e-12, 1.0 / np.sqrt(np.maximum(var, 1e-300)), 0.0)
    mean, inv = mean.astype(np.float32), inv.astype(np.float32)
    net = rt.MLP(seed=5)
    net.set_input_norm(mean, inv)
    X = rt.closure_normalize(feat, mean, inv)
    Y = net.forward(X)
    plain = rt.compute_J_direct(model, d8, chi, eta, m.freq.len, m.freq.dx, I_bc).cpu().numpy()
    sd = np.exp(0.5 * Y[:, 1].reshape(m.P, m.F).max(1).values.double().cpu().numpy())
    solve_bytes = rt.compute_J_workspace(d8, 400, m.F)
    for lb in (float("inf"), float("-inf"), float(np.log(np.quantile(sd, 0.8)))):
        Jref, fl, nf = rt.closure_apply(J1, Y, lb)
        k = int(nf.item())
        if k:
            fine = rt.compute_J_direct(model, d8, chi, eta, m.freq.len, m.freq.dx, I_bc, origins=fl[:k].contiguous())
            rt.closure_merge(fine, fl, k, Jref)
        J, fl2, k2 = rt.closure_J(model, d1, d8, chi, eta, m.freq.len, m.freq.dx, m.freq.x0, I_bc, net, lb,
                                  solve_bytes)
        rt.sync_status()
        assert k2 == k
        assert np.array_equal(np.sort(fl2[:k2].cpu().numpy()), np.sort(fl[:k].cpu().numpy()))
        assert np.array_equal(J.cpu().numpy(), Jref.cpu().numpy())
        if lb == float("-inf"):
            assert k2 == m.P and np.array_equal(J.cpu().numpy(), plain)
