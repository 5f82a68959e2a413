"""ctypes binding of librtmi.so (include/rt.h), marshalling torch tensors."""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtmi.so")

RT_F32 = 1
RT_F64 = 2
SCHED_DIRECT = 0
SCHED_BINNED = 1
SCHED_SPATIAL = 2
MAX_FREQ_BLOCKS = 8

_i32, _i64, _vp, _sz, _dbl = C.c_int32, C.c_int64, C.c_void_p, C.c_size_t, C.c_double
_lib = None


class RtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rt error {code}: {msg}")
        self.code = code


class FreqGridC(C.Structure):
    _fields_ = [("n_blocks", _i32), ("len", C.POINTER(_i32)), ("dx", C.POINTER(_dbl))]


class SolveOptsC(C.Structure):
    _fields_ = [("precision", _i32), ("schedule", _i32), ("dtau_fp64_below", _dbl),
                ("waves_per_cu", _i32), ("n_bins", _i32), ("group", _i32), ("trace_lanes", _i32),
                ("padded_trace_budget", _i64)]


# name -> (restype, argtypes)
_SIGS = {
    "rt_last_error": (C.c_char_p, []),
    "rt_version": (_i32, [C.POINTER(_i32), C.POINTER(_i32)]),
    "rt_dirset_uniform": (_i32, [_i32, C.POINTER(_vp)]),
    "rt_dirset_adaptive": (_i32, [_vp, _i32, _i32, _vp, _i64, _vp, _i64, _vp, C.POINTER(_vp)]),
    "rt_dirset_info": (_i32, [_vp, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i32), C.POINTER(_i32)]),
    "rt_dirset_export": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "rt_dirset_destroy": (_i32, [_vp]),
    "rt_model_create": (_i32, [_vp, _i64, _vp, _vp, _i64, _vp, _vp, C.POINTER(_vp)]),
    "rt_model_destroy": (_i32, [_vp]),
    "rt_validate_host": (_i32, [_vp, _i64, _vp, _vp, _i64, _vp, _i32, _i64, _i64]),
    "rt_trace_count_workspace": (_i32, [_vp, _i64, C.POINTER(_sz)]),
    "rt_trace_count": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _sz, _vp]),
    "rt_trace_write": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _i64, _vp]),
    "rt_solve_workspace": (_i32, [_vp, _i64, _i64, C.POINTER(SolveOptsC), C.POINTER(_sz)]),
    "rt_solve": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _i64, C.POINTER(FreqGridC),
                        _vp, _vp, _vp, C.POINTER(SolveOptsC), _vp, _sz, _vp]),
    "rt_plan_create": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _i32, _i64, C.POINTER(FreqGridC), _vp, _vp,
                              C.POINTER(SolveOptsC), _vp, C.POINTER(_vp)]),
    "rt_plan_run": (_i32, [_vp, _i32, _vp]),
    "rt_plan_info": (_i32, [_vp, C.POINTER(_i64), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp)]),
    "rt_plan_copy_rays": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "rt_plan_profile": (_i32, [_vp, _i32, _vp, _vp]),
    "rt_plan_destroy": (_i32, [_vp]),
    "rt_autotune": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _i32, _i64, C.POINTER(FreqGridC), _vp, _vp,
                           C.POINTER(SolveOptsC), _i32, C.c_char_p, _i32, _vp, C.POINTER(SolveOptsC),
                           C.POINTER(_dbl)]),
    "rt_plan_retune": (_i32, [_vp, C.POINTER(SolveOptsC), _vp]),
    "rt_sync_status": (_i32, [_vp]),
}


def declared_symbols() -> list:
    return list(_SIGS)


def load():
    """Load librtmi.so (built by __graft_entry__.build() / paper_2011_14998_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RtError(-5, f"{LIB_PATH} is not built; run paper_2011_14998_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code != 0:
        raise RtError(code, load().rt_last_error().decode())


def version():
    a, b = _i32(), _i32()
    _check(load().rt_version(C.byref(a), C.byref(b)))
    return a.value, b.value


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dev(t, dtype):
    torch = _torch()
    assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), (t.device, t.dtype)
    return t


class DirSet:
    """A HEALPix direction set handle (uniform or adaptive)."""

    def __init__(self, handle, keep=()):
        self._h = C.c_void_p(handle)
        self._keep = keep

    @classmethod
    def uniform(cls, nside: int) -> "DirSet":
        h = _vp()
        _check(load().rt_dirset_uniform(nside, C.byref(h)))
        return cls(h.value)

    @classmethod
    def adaptive(cls, model: "Model", lmin: int, lmax: int, sample_ids, origins=None, n_origins=None,
                 stream=None) -> "DirSet":
        torch = _torch()
        sample_ids = _dev(sample_ids, torch.int32)
        if origins is not None:
            origins = _dev(origins, torch.int32)
            n_origins = origins.numel()
        elif n_origins is None:
            n_origins = model.P
        h = _vp()
        _check(load().rt_dirset_adaptive(model._h, lmin, lmax, _ptr(sample_ids), sample_ids.numel(),
                                         _ptr(origins), n_origins, _stream(stream), C.byref(h)))
        return cls(h.value, keep=(sample_ids, origins))

    def info(self):
        R, n, lo, hi = _i64(), _i64(), _i32(), _i32()
        _check(load().rt_dirset_info(self._h, C.byref(R), C.byref(n), C.byref(lo), C.byref(hi)))
        return dict(R=R.value, n_origins=n.value, lmin=lo.value, lmax=hi.value)

    @property
    def R(self) -> int:
        return self.info()["R"]

    def export(self, stream=None):
        inf = self.info()
        n = max(1, inf["n_origins"])
        R = inf["R"]
        pix = np.zeros((n, R), np.int64)
        lev = np.zeros((n, R), np.int32)
        dirs = np.zeros((n, R, 3))
        w2 = np.zeros((n, R))
        s = _stream(stream) if inf["n_origins"] > 0 else None
        _check(load().rt_dirset_export(self._h, pix.ctypes.data, lev.ctypes.data, dirs.ctypes.data,
                                       w2.ctypes.data, s))
        if inf["n_origins"] == 0:
            return pix[0], lev[0], dirs[0], w2[0]
        return pix, lev, dirs, w2

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None):
            _lib.rt_dirset_destroy(self._h)
            self._h = None


class Model:
    """Device-resident point cloud + neighbour lists (+ optional velocities)."""

    def __init__(self, pos, nbr_off, nbr_idx, vel=None, stream=None):
        torch = _torch()
        self.pos = _dev(pos, torch.float64)
        self.nbr_off = _dev(nbr_off, torch.int64)
        self.nbr_idx = _dev(nbr_idx, torch.int32)
        self.vel = None if vel is None else _dev(vel, torch.float32)
        self.P = self.pos.shape[0]
        h = _vp()
        _check(load().rt_model_create(_ptr(self.pos), self.P, _ptr(self.nbr_off), _ptr(self.nbr_idx),
                                      self.nbr_idx.numel(), _ptr(self.vel), _stream(stream), C.byref(h)))
        self._h = h

    @classmethod
    def from_numpy(cls, pos, nbr_off, nbr_idx, vel=None, device="cuda"):
        torch = _torch()
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)  # noqa: E731
        return cls(t(pos, torch.float64), t(nbr_off, torch.int64), t(nbr_idx, torch.int32),
                   None if vel is None else t(vel, torch.float32))

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None):
            _lib.rt_model_destroy(self._h)
            self._h = None


def validate_host(pos, nbr_off, nbr_idx, chi=None, F=0, ld=0):
    """Host-side validation (numpy arrays); raises RtError on the first problem."""
    pos = np.ascontiguousarray(pos, np.float64)
    off = np.ascontiguousarray(nbr_off, np.int64)
    idx = np.ascontiguousarray(nbr_idx, np.int32)
    dt, cp = 0, None
    if chi is not None:
        chi = np.ascontiguousarray(chi)
        dt = RT_F32 if chi.dtype == np.float32 else RT_F64
        F = F or chi.shape[1]
        ld = ld or chi.shape[1]
        cp = chi.ctypes.data
    _check(load().rt_validate_host(pos.ctypes.data, pos.shape[0], off.ctypes.data, idx.ctypes.data, idx.size,
                                   cp, dt, F, ld))


def sync_status(stream=None):
    _check(load().rt_sync_status(_stream(stream)))


def trace(model: Model, dirset: DirSet, origins=None, n_origins=None, stream=None):
    """Ray lists (ray_off int64 [n_o*2R+1], ids int32 [T], Z float64 [T]) as device tensors."""
    torch = _torch()
    L = load()
    if origins is not None:
        origins = _dev(origins, torch.int32)
        n_origins = origins.numel()
    elif n_origins is None:
        n_origins = model.P
    R = dirset.R
    n_rays = n_origins * 2 * R
    s = _stream(stream)
    wsb = _sz()
    _check(L.rt_trace_count_workspace(dirset._h, n_origins, C.byref(wsb)))
    ws = torch.empty(max(1, wsb.value), dtype=torch.uint8, device=model.pos.device)
    ray_off = torch.empty(n_rays + 1, dtype=torch.int64, device=model.pos.device)
    _check(L.rt_trace_count(model._h, dirset._h, _ptr(origins), n_origins, _ptr(ray_off), _ptr(ws), wsb.value, s))
    total = int(ray_off[-1].item())
    ids = torch.empty(max(total, 1), dtype=torch.int32, device=model.pos.device)
    Z = torch.empty(max(total, 1), dtype=torch.float64, device=model.pos.device)
    _check(L.rt_trace_write(model._h, dirset._h, _ptr(origins), n_origins, _ptr(ray_off), _ptr(ids), _ptr(Z),
                            total, s))
    sync_status(stream)
    return ray_off, ids[:total], Z[:total]


def _grid(freq_len: Sequence[int], freq_dx: Sequence[float]):
    ln = (_i32 * len(freq_len))(*[int(x) for x in freq_len])
    dx = (_dbl * len(freq_dx))(*[float(x) for x in freq_dx])
    g = FreqGridC(len(freq_len), ln, dx)
    return g, (ln, dx)


def _opts(precision, schedule, dtau_fp64_below, waves_per_cu, n_bins, padded_trace_budget=0, group=0,
          trace_lanes=0):
    return SolveOptsC(precision, schedule, dtau_fp64_below, waves_per_cu, n_bins, group, trace_lanes,
                      padded_trace_budget)


def solve(model: Model, dirset: DirSet, rays, chi, eta, freq_len, freq_dx, I_bc, origins=None, n_origins=None,
          precision: int = RT_F32, schedule: int = SCHED_DIRECT, dtau_fp64_below: float = 1e-4,
          waves_per_cu: int = 0, n_bins: int = 0, group: int = 0, want_u: bool = False, stream=None):
    """J [n_o][F] (dtype of the precision) from ray lists; optionally u [n_o][R][F]."""
    torch = _torch()
    L = load()
    dt = torch.float64 if precision == RT_F64 else torch.float32
    chi = _dev(chi, dt)
    eta = _dev(eta, dt)
    I_bc = _dev(I_bc, torch.float64)
    if origins is not None:
        origins = _dev(origins, torch.int32)
        n_origins = origins.numel()
    elif n_origins is None:
        n_origins = model.P
    ray_off, ids, Z = rays
    F = int(sum(freq_len))
    R = dirset.R
    g, keep = _grid(freq_len, freq_dx)
    o = _opts(precision, schedule, dtau_fp64_below, waves_per_cu, n_bins, group=group)
    u = torch.empty((n_origins, R, F), dtype=dt, device=chi.device) if want_u else None
    wsb = _sz()
    _check(L.rt_solve_workspace(dirset._h, n_origins, F, C.byref(o), C.byref(wsb)))
    ws = torch.empty(max(1, wsb.value), dtype=torch.uint8, device=chi.device)
    J = torch.empty((n_origins, F), dtype=dt, device=chi.device)
    _check(L.rt_solve(model._h, dirset._h, _ptr(origins), n_origins, _ptr(ray_off), _ptr(ids), _ptr(Z),
                      _ptr(chi), _ptr(eta), precision, chi.shape[1], C.byref(g), _ptr(I_bc), _ptr(J), _ptr(u),
                      C.byref(o), _ptr(ws), wsb.value, _stream(stream)))
    sync_status(stream)
    del keep
    return (J, u) if want_u else J


def compute_J(model: Model, dirset: DirSet, chi, eta, freq_len, freq_dx, I_bc, origins=None, **kw):
    rays = trace(model, dirset, origins=origins)
    return solve(model, dirset, rays, chi, eta, freq_len, freq_dx, I_bc, origins=origins, **kw)


def autotune(model: Model, dirset: DirSet, chi, eta, freq_len, freq_dx, I_bc, J, origins=None, n_origins=None,
             precision: int = RT_F32, dtau_fp64_below: float = 1e-4, n_runs: int = 2, cache_path: str = None,
             verbose: bool = False, stream=None):
    """Fastest plan options for this workload (see rt_autotune); returns (options dict, ms per step)."""
    torch = _torch()
    dt = torch.float64 if precision == RT_F64 else torch.float32
    chi, eta, J = _dev(chi, dt), _dev(eta, dt), _dev(J, dt)
    I_bc = _dev(I_bc, torch.float64)
    if origins is not None:
        origins = _dev(origins, torch.int32)
        n_origins = origins.numel()
    elif n_origins is None:
        n_origins = model.P
    g, keep = _grid(freq_len, freq_dx)
    base = _opts(precision, SCHED_SPATIAL, dtau_fp64_below, 0, 0)
    best = SolveOptsC()
    ms = _dbl()
    _check(load().rt_autotune(model._h, dirset._h, _ptr(origins), n_origins, _ptr(chi), _ptr(eta), precision,
                              chi.shape[1], C.byref(g), _ptr(I_bc), _ptr(J), C.byref(base), n_runs,
                              None if cache_path is None else cache_path.encode(), 1 if verbose else 0,
                              _stream(stream), C.byref(best), C.byref(ms)))
    del keep
    opts = dict(schedule=best.schedule, group=best.group, trace_lanes=best.trace_lanes,
                waves_per_cu=best.waves_per_cu, n_bins=best.n_bins)
    return opts, ms.value


class Plan:
    """The whole hot path (count, scan, write, bin, sweep, reduce) as one replayable HIP graph."""

    def __init__(self, model: Model, dirset: DirSet, chi, eta, freq_len, freq_dx, I_bc, J, origins=None,
                 n_origins=None, precision: int = RT_F32, schedule: int = SCHED_DIRECT,
                 dtau_fp64_below: float = 1e-4, waves_per_cu: int = 0, n_bins: int = 0,
                 padded_trace_budget: int = 0, group: int = 0, trace_lanes: int = 0, stream=None):
        torch = _torch()
        dt = torch.float64 if precision == RT_F64 else torch.float32
        self.chi, self.eta, self.J = _dev(chi, dt), _dev(eta, dt), _dev(J, dt)
        self.I_bc = _dev(I_bc, torch.float64)
        if origins is not None:
            origins = _dev(origins, torch.int32)
            n_origins = origins.numel()
        elif n_origins is None:
            n_origins = model.P
        self.origins, self.n_origins = origins, n_origins
        self.model, self.dirset = model, dirset
        g, self._keep = _grid(freq_len, freq_dx)
        o = _opts(precision, schedule, dtau_fp64_below, waves_per_cu, n_bins, padded_trace_budget, group, trace_lanes)
        h = _vp()
        _check(load().rt_plan_create(model._h, dirset._h, _ptr(origins), n_origins, _ptr(self.chi),
                                     _ptr(self.eta), precision, self.chi.shape[1], C.byref(g), _ptr(self.I_bc),
                                     _ptr(self.J), C.byref(o), _stream(stream), C.byref(h)))
        self._h = h

    def retune(self, schedule: int = SCHED_SPATIAL, group: int = 0, trace_lanes: int = 0, waves_per_cu: int = 0,
               n_bins: int = 0, stream=None):
        """Re-capture the plan's graph with other scheduling options."""
        o = _opts(RT_F32, schedule, 1e-4, waves_per_cu, n_bins, 0, group, trace_lanes)
        _check(load().rt_plan_retune(self._h, C.byref(o), _stream(stream)))

    def run(self, use_graph: bool = True, stream=None):
        _check(load().rt_plan_run(self._h, 1 if use_graph else 0, _stream(stream)))

    STAGES = ("walk", "scan", "lists", "bin", "sweep", "reduce")

    def profile(self, n_runs: int, stream=None) -> dict:
        """Mean per-stage times (ms) over n_runs eager runs, from HIP events on the stream."""
        out = np.zeros(6)
        _check(load().rt_plan_profile(self._h, n_runs, out.ctypes.data, _stream(stream)))
        return dict(zip(self.STAGES, out.tolist()))

    def info(self):
        tot = _i64()
        off, ids, Z = _vp(), _vp(), _vp()
        _check(load().rt_plan_info(self._h, C.byref(tot), C.byref(off), C.byref(ids), C.byref(Z)))
        return dict(total=tot.value, ray_off=off.value, ray_ids=ids.value, ray_Z=Z.value)

    def rays(self, stream=None):
        """Copies of the plan's ray lists (ray_off, ids, Z) as device tensors."""
        torch = _torch()
        tot = self.info()["total"]
        n = self.n_origins * 2 * self.dirset.R + 1
        dev = self.J.device
        off = torch.empty(n, dtype=torch.int64, device=dev)
        ids = torch.empty(max(tot, 1), dtype=torch.int32, device=dev)
        Z = torch.empty(max(tot, 1), dtype=torch.float64, device=dev)
        _check(load().rt_plan_copy_rays(self._h, _ptr(off), _ptr(ids), _ptr(Z), _stream(stream)))
        return off, ids[:tot], Z[:tot]

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None):
            _lib.rt_plan_destroy(self._h)
            self._h = None
