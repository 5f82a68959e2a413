"""Tables whose byte offsets exceed 32 bits take the sweep's other addressing
path (the row moved to scalar registers per point instead of a 32-bit lane
offset): the same model solved from such tables -- the same values at a row
stride of several million entries -- gives J bit-identical to the compact
tables, moving and static, uniform and per-block frequency widths, FP32 and
FP64."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "moving":
        return synth.tiny_model(71, P=120, F=16, moving=True)
    if name == "static":
        return synth.tiny_model(72, P=120, F=16, moving=False)
    m = synth.tiny_model(73, P=120, F=20, moving=True)  # per-lane widths: blocks of different dx
    m.freq = synth.FreqGrid(np.array([12, 8], np.int32), np.array([-3.0, -2.0]), np.array([0.5, 0.6]))
    return m


@pytest.mark.parametrize("name", ["moving", "static", "blocks"])
@pytest.mark.parametrize("fp64", [False, True])
def test_wide_tables_bit_identical(rt, name, fp64):
    import torch
    m = _case(name)
    dt = torch.float64 if fp64 else torch.float32
    prec = rt.RT_F64 if fp64 else rt.RT_F32
    es = 8 if fp64 else 4
    model = rt.Model.from_numpy(m.pos, m.nbr_off, m.nbr_idx, m.vel)
    ds = rt.DirSet.uniform(1)
    rays = rt.trace(model, ds)
    chi = torch.as_tensor(m.chi, dtype=dt, device="cuda").contiguous()
    eta = torch.as_tensor(m.eta, dtype=dt, device="cuda").contiguous()
    I_bc = torch.as_tensor(m.I_bc, dtype=torch.float64, device="cuda")
    J0 = rt.solve(model, ds, rays, chi, eta, m.freq.len, m.freq.dx, I_bc, precision=prec).cpu().numpy()
    ld = (1 << 32) // (m.P * es) + 64  # P * ld * es > 4 GiB
    print(f"{name} fp64={fp64}: ld {ld}, {m.P * ld * es / 2**30:.2f} GiB per table", flush=True)
    chw, etw = _wide(chi, ld), _wide(eta, ld)
    J1 = rt.solve(model, ds, rays, chw, etw, m.freq.len, m.freq.dx, I_bc, precision=prec).cpu().numpy()
    del chw, etw
    torch.cuda.empty_cache()
    assert np.array_equal(J0, J1)


def _wide(t, ld):
    import torch
    w = torch.zeros((t.shape[0], ld), dtype=t.dtype, device=t.device)
    w[:, :t.shape[1]] = t
    return w
