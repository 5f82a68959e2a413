"""rt_solve_noalloc (the solve on the library's static scratch) against rt_solve (the
same solve on a caller workspace), through the C ABI: two calls in a row, the second on
a smaller input, so the second call runs on scratch the first one left behind.  Bit for
bit in FP32 and FP64, direct and length-binned; sizes beyond the scratch are rejected
before anything is launched; and the call allocates no device memory."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("schedule", ["direct", "binned"])
@pytest.mark.parametrize("fp64", [False, True])
def test_noalloc_matches_solve_twice(rt, schedule, fp64):
    import torch
    sc = rt.SCHED_BINNED if schedule == "binned" else rt.SCHED_DIRECT
    prec = rt.RT_F64 if fp64 else rt.RT_F32
    dt = np.float64 if fp64 else np.float32
    m = synth.wind_model(seed=6, P=6000)
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    ds = rt.DirSet.uniform(2)
    chi, eta = _t(m.chi.astype(dt)), _t(m.eta.astype(dt))
    I_bc = _t(m.I_bc, torch.float64)
    rng = np.random.default_rng(9)
    for n in (2500, 700):  # the second call is smaller and reuses the first call's scratch
        org = _t(rng.permutation(m.P)[:n].astype(np.int32))
        rays = rt.trace(model, ds, origins=org)
        ref = rt.solve(model, ds, rays, chi, eta, m.freq.len, m.freq.dx, I_bc, origins=org, precision=prec,
                       schedule=sc).cpu().numpy()
        J = torch.full((n, m.F), -1.0, dtype=chi.dtype, device="cuda")
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        rt.solve_noalloc(model, ds, rays, chi, eta, m.freq.len, m.freq.dx, I_bc, J, origins=org, precision=prec,
                         schedule=sc)
        rt.sync_status()
        assert torch.cuda.memory_allocated() == before
        assert np.array_equal(J.cpu().numpy(), ref), n


def test_noalloc_u_out_and_limit(rt):
    """With u_out the scratch holds only the bins, so a call too large for the scratch
    without it runs with it; the too-large call is refused with RT_ERR_CAPACITY."""
    import torch
    m = synth.wind_model(seed=7, P=8000)
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    ds = rt.DirSet.uniform(4)  # 96 pairs: u of 8000 origins is 8000*96*64*4 B = 197 MB > 64 MiB
    c32, e32, _, _ = synth.to_fp32_tables(m.chi, m.eta)
    chi, eta, I_bc = _t(c32), _t(e32), _t(m.I_bc, torch.float64)
    rays = rt.trace(model, ds)
    J = torch.empty((m.P, m.F), dtype=torch.float32, device="cuda")
    with pytest.raises(rt.RtError) as e:
        rt.solve_noalloc(model, ds, rays, chi, eta, m.freq.len, m.freq.dx, I_bc, J)
    assert e.value.code == -4 and "64 MiB" in str(e.value)
    u = torch.empty((m.P, ds.R, m.F), dtype=torch.float32, device="cuda")
    rt.solve_noalloc(model, ds, rays, chi, eta, m.freq.len, m.freq.dx, I_bc, J, u=u, schedule=rt.SCHED_BINNED)
    rt.sync_status()
    ref, uref = rt.solve(model, ds, rays, chi, eta, m.freq.len, m.freq.dx, I_bc, want_u=True)
    assert np.array_equal(J.cpu().numpy(), ref.cpu().numpy())
    assert np.array_equal(u.cpu().numpy(), uref.cpu().numpy())
