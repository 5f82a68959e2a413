"""GPU parity at full size: the launch shapes the benchmark times and the paths only large
inputs reach, checked against the oracle on seeded samples of origins.

- 64 SPH-like clouds, 4.1 million particles, as one device-built union (rt_batch, each
  model's points renumbered into Morton order; lists compared through the union index), nside
  2, F = 64: the walk (8 lanes per ray, 197 million rays) and the sweep (spatial direct launch,
  98 million items) both need more workgroups than one dispatch takes, so both run their
  grid-stride rounds.
- The AMR-octree-like cloud at about 500 000 leaves, nside 4, F = 96 in two lines of 48
  (each pair takes a 64-lane chunk and a 32-lane chunk), 16 lanes per ray: grid-stride rounds
  in walk and sweep.
- rt_compute_J on a 500 000-point wind at nside 8 in a workspace that forces tens of
  Morton-ordered chunks (the closure's label and fallback path).

Bars: sampled ray lists bit-exact (ids and the bits of Z), sampled J within 1e-4 of the FP64
oracle fed the same FP32 tables."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-4


def _torch():
    import torch
    return torch


def _t(a, dtype=None):
    torch = _torch()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


def _sampled_rays(views, slots_of, origins, two_r):
    """(offsets, ids, Z) of the listed origins' 2R rays, gathered on the device from lists
    that are too large to copy whole; offsets restarted at 0 like the oracle's."""
    torch = _torch()
    off, ids, Z = views
    out_off, out_ids, out_Z = [0], [], []
    for o in origins:
        s0 = int(slots_of(o))
        o_off = off[s0:s0 + two_r + 1].cpu().numpy()
        lo, hi = int(o_off[0]), int(o_off[-1])
        out_ids.append(ids[lo:hi].cpu().numpy())
        out_Z.append(Z[lo:hi].cpu().numpy())
        out_off.extend((o_off[1:] - lo + out_off[-1]).tolist())
    torch.cuda.synchronize()
    return np.array(out_off, np.int64), np.concatenate(out_ids), np.concatenate(out_Z)


def _assert_rays(g, e, id_shift=0):
    assert np.array_equal(g[0], e[0])
    assert np.array_equal(g[1], e[1].astype(np.int64) + id_shift)
    assert np.array_equal(g[2].view(np.uint64), e[2].view(np.uint64))


def test_sph_batch_full_size(rt, orc):
    torch = _torch()
    ms = synth.sph_batch_models(n_models=64, scale=1.0, workers=16)
    P_tot = sum(m.P for m in ms)
    assert P_tot > 4_000_000
    models, chis, etas, Js = [], [], [], []
    for m in ms:
        c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
        models.append(rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel))
        chis.append(_t(c32))
        etas.append(_t(e32))
        Js.append(torch.empty((m.P, m.F), dtype=torch.float32, device="cuda"))
    ds = rt.DirSet.uniform(2)
    two_r = 2 * ds.R
    b = rt.Batch(models, ds, chis, etas, ms[0].freq.len, ms[0].freq.dx, _t(ms[0].I_bc, torch.float64), Js,
                 schedule=rt.SCHED_SPATIAL, trace_lanes=8)
    # grid-stride rounds are reached: both launches need more than 2^22 workgroups
    assert P_tot * two_r * 8 // 256 > (1 << 22) and P_tot * ds.R // 4 > (1 << 22)
    b.run()
    rt.sync_status()
    print(f"union of {P_tot} particles, {b.info()['total']} list entries", flush=True)
    _, dirs, w2 = orc.dirset_uniform(2)
    views = b.rays_view()
    uidx = b.union_index().cpu().numpy().astype(np.int64)  # union id of model point base_k + i
    rng = np.random.default_rng(40)
    base = np.concatenate([[0], np.cumsum([m.P for m in ms])])
    checked = 0
    for k in rng.choice(64, 12, replace=False):
        m = ms[k]
        local = np.sort(rng.choice(m.P, 25, replace=False)).astype(np.int32)
        if k == 0:
            local[0] = 0
        g = _sampled_rays(views, lambda o: uidx[base[k] + o] * two_r, local, two_r)
        e = orc.trace_all(m, dirs, local)
        _assert_rays(g, (e[0], uidx[base[k] + e[1].astype(np.int64)], e[2]))
        c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
        Je = orc.compute_J(m, dirs, w2, origins=local, chi=c64, eta=e64)
        assert _rel(Js[k][_t(local).long()].cpu().numpy().astype(np.float64), Je) <= TOL32
        checked += len(local)
    assert checked == 300


def test_octree_full_size_two_chunks(rt, orc):
    torch = _torch()
    m = synth.octree_model(seed=3, target=500_000)
    assert m.F == 96 and m.P > 490_000
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    ds = rt.DirSet.uniform(4)
    two_r = 2 * ds.R
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    J = torch.empty((m.P, m.F), dtype=torch.float32, device="cuda")
    plan = rt.Plan(model, ds, _t(c32), _t(e32), m.freq.len, m.freq.dx, _t(m.I_bc, torch.float64), J,
                   n_origins=m.P, precision=rt.RT_F32, schedule=rt.SCHED_SPATIAL, trace_lanes=16)
    assert m.P * two_r * 16 // 256 > (1 << 22) and m.P * ds.R * 2 // 4 > (1 << 22)
    plan.run()
    rt.sync_status()
    print(f"octree of {m.P} leaves, {plan.info()['total']} list entries", flush=True)
    rng = np.random.default_rng(41)
    sample = np.sort(rng.choice(m.P, 300, replace=False)).astype(np.int32)
    sample[-1] = m.P - 1
    g = _sampled_rays(plan.rays_view(), lambda o: o * two_r, sample, two_r)
    _, dirs, w2 = orc.dirset_uniform(4)
    _assert_rays(g, orc.trace_all(m, dirs, sample))
    Je = orc.compute_J(m, dirs, w2, origins=sample, chi=c64, eta=e64)
    got = J[_t(sample).long()].cpu().numpy().astype(np.float64)
    assert _rel(got, Je) <= TOL32
    # both frequency chunks of a pair: the lanes of the second line (64..95) as well as the first
    assert _rel(got[:, 64:], Je[:, 64:]) <= TOL32 and _rel(got[:, :48], Je[:, :48]) <= TOL32


def test_compute_J_wind_nside8_chunked(rt, orc):
    torch = _torch()
    m = synth.wind_model(seed=510, P=500_000)
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    ds = rt.DirSet.uniform(8)
    c32, e32, c64, e64 = synth.to_fp32_tables(m.chi, m.eta)
    rng = np.random.default_rng(42)
    origins = rng.permutation(m.P)[:40_000].astype(np.int32)
    ws = rt.compute_J_workspace(ds, len(origins), m.F) // 40  # tens of chunks
    J = rt.compute_J(model, ds, _t(c32), _t(e32), m.freq.len, m.freq.dx, _t(m.I_bc, torch.float64),
                     origins=_t(origins), ws_bytes=ws)
    rt.sync_status()
    pick = np.sort(rng.choice(len(origins), 60, replace=False))
    _, dirs, w2 = orc.dirset_uniform(8)
    Je = orc.compute_J(m, dirs, w2, origins=origins[pick], chi=c64, eta=e64)
    assert _rel(J.cpu().numpy()[pick].astype(np.float64), Je) <= TOL32
