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
SCHEME_FEAUTRIER2 = 0
SCHEME_HERMITE = 1
WALK_EXACT = 0
WALK_PADDED = 1
WALK_TWO_PASS = 2
MAX_FREQ_BLOCKS = 8

_i32, _i64, _vp, _sz, _dbl = C.c_int32, C.c_int64, C.c_void_p, C.c_size_t, C.c_double
_lib = None


class RtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rt error {code}: {msg}")
        self.code = code


class FreqGridC(C.Structure):
    _fields_ = [("n_blocks", _i32), ("len", C.POINTER(_i32)), ("dx", C.POINTER(_dbl)), ("x0", C.POINTER(_dbl))]


class SolveOptsC(C.Structure):
    _fields_ = [("precision", _i32), ("schedule", _i32),
                ("waves_per_cu", _i32), ("n_bins", _i32), ("bins_per_octave", _i32), ("group", _i32),
                ("trace_lanes", _i32), ("padded_trace_budget", _i64), ("walk", _i32), ("dtau_max", _dbl),
                ("max_substeps", _i32), ("dv_max", _dbl), ("scheme", _i32)]


class TrainOptsC(C.Structure):
    _fields_ = [("batch", _i64), ("total_steps", _i64), ("lr", C.c_float), ("lr_final", C.c_float),
                ("b1", C.c_float), ("b2", C.c_float), ("eps", C.c_float), ("wd", C.c_float), ("seed", C.c_uint64)]


# name -> (restype, argtypes)
_SIGS = {
    "rt_last_error": (C.c_char_p, []),
    "rt_version": (_i32, [C.POINTER(_i32), C.POINTER(_i32)]),
    "rt_struct_sizes": (_i32, [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
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
    "rt_trace": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _i64, _vp, _vp, _sz, _vp]),
    "rt_solve_workspace": (_i32, [_vp, _i64, _i64, C.POINTER(SolveOptsC), C.POINTER(_sz)]),
    "rt_solve": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _i64, C.POINTER(FreqGridC),
                        _vp, _vp, _vp, C.POINTER(SolveOptsC), _vp, _sz, _vp]),
    "rt_solve_noalloc": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _i32, _i64, C.POINTER(FreqGridC),
                                _vp, _vp, _vp, C.POINTER(SolveOptsC), _vp]),
    "rt_plan_create": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _i32, _i64, C.POINTER(FreqGridC), _vp, _vp,
                              C.POINTER(SolveOptsC), _vp, C.POINTER(_vp)]),
    "rt_plan_run": (_i32, [_vp, _i32, _vp]),
    "rt_plan_info": (_i32, [_vp, C.POINTER(_i64), C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp)]),
    "rt_plan_copy_rays": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "rt_plan_profile": (_i32, [_vp, _i32, _vp, _vp]),
    "rt_plan_destroy": (_i32, [_vp]),
    "rt_release_cached_memory": (_i32, []),
    "rt_cached_memory": (_i32, [C.POINTER(C.c_size_t)]),
    "rt_plan_memory": (_i32, [C.POINTER(C.c_size_t)]),
    "rt_autotune": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _i32, _i64, C.POINTER(FreqGridC), _vp, _vp,
                           C.POINTER(SolveOptsC), _i32, C.c_char_p, _i32, _vp, C.POINTER(SolveOptsC),
                           C.POINTER(_dbl)]),
    "rt_plan_retune": (_i32, [_vp, C.POINTER(SolveOptsC), _vp]),
    "rt_autotune_plan": (_i32, [_vp, _i32, _i32, _vp, C.POINTER(SolveOptsC), C.POINTER(_dbl)]),
    "rt_compute_J_workspace": (_i32, [_vp, _i64, _i64, C.POINTER(SolveOptsC), _dbl, C.POINTER(_sz)]),
    "rt_compute_J": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _i32, _i64, C.POINTER(FreqGridC), _vp, _vp, _vp,
                            C.POINTER(SolveOptsC), _vp, _sz, _vp]),
    "rt_batch_create": (_i32, [_i32, _vp, _vp, _vp, _vp, _i32, _vp, C.POINTER(FreqGridC), _vp, _vp,
                               C.POINTER(SolveOptsC), _vp, C.POINTER(_vp)]),
    "rt_batch_run": (_i32, [_vp, _i32, _vp]),
    "rt_batch_plan": (_i32, [_vp, C.POINTER(_vp)]),
    "rt_batch_union": (_i32, [_vp, C.POINTER(_i64), C.POINTER(_i64)]),
    "rt_batch_union_index": (_i32, [_vp, _vp, _vp]),
    "rt_batch_destroy": (_i32, [_vp]),
    "rt_compute_J_batched": (_i32, [_i32, _vp, _vp, _vp, _vp, _i32, _vp, C.POINTER(FreqGridC), _vp, _vp,
                                    C.POINTER(SolveOptsC), _vp]),
    "rt_mlp_set_input_norm": (_i32, [_vp, _vp, _vp]),
    "rt_closure_J_workspace": (_i32, [_vp, _vp, _i64, _sz, C.POINTER(_sz)]),
    "rt_closure_J": (_i32, [_vp, _vp, _vp, _vp, _vp, _i64, C.POINTER(FreqGridC), _vp, _vp, C.c_float, _vp, _vp,
                            C.POINTER(_i64), C.POINTER(SolveOptsC), _vp, _sz, _vp]),
    "rt_sync_status": (_i32, [_vp]),
    "rt_mlp_num_params": (_i32, [C.POINTER(_i64)]),
    "rt_mlp_create": (_i32, [C.c_uint64, _vp, C.POINTER(_vp)]),
    "rt_mlp_destroy": (_i32, [_vp]),
    "rt_mlp_get_params": (_i32, [_vp, _vp, _vp]),
    "rt_mlp_set_params": (_i32, [_vp, _vp, _vp]),
    "rt_mlp_get_grads": (_i32, [_vp, _vp, _vp]),
    "rt_mlp_zero_grad": (_i32, [_vp, _vp]),
    "rt_mlp_workspace": (_i32, [_i64, _i32, C.POINTER(_sz)]),
    "rt_mlp_forward": (_i32, [_vp, _vp, _vp, _i64, _vp, _i32, _vp, _sz, _vp]),
    "rt_mlp_backward": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _sz, _vp]),
    "rt_mlp_nll": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "rt_mlp_adam_step": (_i32, [_vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float, _vp]),
    "rt_mlp_train_workspace": (_i32, [_i64, C.POINTER(_sz)]),
    "rt_mlp_train": (_i32, [_vp, _vp, _vp, _i64, C.POINTER(TrainOptsC), _i64, _vp, _vp, _sz, _vp]),
    "rt_closure_features": (_i32, [_vp, _vp, _vp, _i64, _i64, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp]),
    "rt_plan_copy_u": (_i32, [_vp, _vp, _vp]),
    "rt_spatial_order": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "rt_mesh_indicators": (_i32, [_vp, _vp, _dbl, _dbl, _dbl, _vp, _vp, _vp, _vp]),
    "rt_healpix_vec2pix": (_i32, [_i32, _vp, _i64, _vp]),
    "rt_closure_feature_stats": (_i32, [_vp, _i64, _vp, _vp, _vp]),
    "rt_closure_normalize": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp]),
    "rt_closure_apply": (_i32, [_vp, _vp, _i64, _i64, C.c_float, _vp, _vp, _vp, _vp]),
    "rt_closure_merge": (_i32, [_vp, _vp, _i64, _i64, _i64, _vp, _vp]),
    "rt_closure_targets": (_i32, [_vp, _vp, _i64, _vp, _vp]),
}


def declared_symbols() -> list:
    return list(_SIGS)


def load():
    """Load librtmi.so (built by __graft_entry__.build() / paper_2011_14998_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RtError(-5, f"{LIB_PATH} is not built; run paper_2011_14998_amd/build.py")
        # torch first: its HIP runtime is the one the process uses (device memory and streams come
        # from torch), and the library must bind to that runtime rather than load one of its own
        _torch()
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


class _DevArray:
    """Library-owned device memory described for torch.as_tensor (zero copy)."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 2}


def _view(ptr: int, n: int, typestr: str):
    """A torch tensor aliasing n elements of library-owned device memory at ptr (no copy); valid
    while the owning handle lives."""
    torch = _torch()
    return torch.as_tensor(_DevArray(ptr, max(n, 0), typestr), device="cuda")


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


def spatial_order(model: Model, origins=None, n_origins=None, stream=None) -> np.ndarray:
    """Positions of the origin list in Morton order of the origins' coordinates (host int32)."""
    torch = _torch()
    if origins is not None:
        origins = _dev(origins, torch.int32)
        n_origins = origins.numel()
    elif n_origins is None:
        n_origins = model.P
    out = np.empty(max(n_origins, 1), np.int32)
    _check(load().rt_spatial_order(model._h, _ptr(origins), n_origins, out.ctypes.data, _stream(stream)))
    return out[:n_origins]


def release_cached_memory():
    """Free the device buffers that destroyed plans left in the library's cache."""
    _check(load().rt_release_cached_memory())


def cached_memory() -> int:
    """Bytes of device memory held by the library's cache of plan buffers."""
    b = _sz()
    _check(load().rt_cached_memory(C.byref(b)))
    return int(b.value)


def plan_memory() -> int:
    """Bytes of the large plan buffers owned by plans not yet destroyed."""
    b = _sz()
    _check(load().rt_plan_memory(C.byref(b)))
    return int(b.value)


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


def trace_once(model: Model, dirset: DirSet, capacity: int, origins=None, n_origins=None, stream=None):
    """rt_trace: count, scan and write in one call into lists of `capacity` entries; returns
    (ray_off, ids, Z, total) with total read back (the lists are complete when total <= capacity)."""
    torch = _torch()
    L = load()
    if origins is not None:
        origins = _dev(origins, torch.int32)
        n_origins = origins.numel()
    elif n_origins is None:
        n_origins = model.P
    dev = model.pos.device
    wsb = _sz()
    _check(L.rt_trace_count_workspace(dirset._h, n_origins, C.byref(wsb)))
    ws = torch.empty(max(1, wsb.value), dtype=torch.uint8, device=dev)
    ray_off = torch.empty(n_origins * 2 * dirset.R + 1, dtype=torch.int64, device=dev)
    ids = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    Z = torch.empty(max(capacity, 1), dtype=torch.float64, device=dev)
    total = torch.empty(1, dtype=torch.int64, device=dev)
    _check(L.rt_trace(model._h, dirset._h, _ptr(origins), n_origins, _ptr(ray_off), _ptr(ids), _ptr(Z), capacity,
                      _ptr(total), _ptr(ws), wsb.value, _stream(stream)))
    return ray_off, ids, Z, int(total.item())


def _grid(freq_len: Sequence[int], freq_dx: Sequence[float], freq_x0: Sequence[float] = None):
    ln = (_i32 * len(freq_len))(*[int(x) for x in freq_len])
    dx = (_dbl * len(freq_dx))(*[float(x) for x in freq_dx])
    x0 = None if freq_x0 is None else (_dbl * len(freq_x0))(*[float(x) for x in freq_x0])
    g = FreqGridC(len(freq_len), ln, dx, x0)
    return g, (ln, dx, x0)


def _opts(precision=RT_F32, schedule=0, waves_per_cu=0, n_bins=0, padded_trace_budget=0, group=0,
          trace_lanes=0, walk=0, dtau_max=0.0, max_substeps=0, dv_max=0.0, scheme=0, bins_per_octave=0):
    return SolveOptsC(precision=precision, schedule=schedule, waves_per_cu=waves_per_cu, n_bins=n_bins,
                      bins_per_octave=bins_per_octave, group=group, trace_lanes=trace_lanes,
                      padded_trace_budget=padded_trace_budget, walk=walk, dtau_max=dtau_max,
                      max_substeps=max_substeps, dv_max=dv_max, scheme=scheme)


def opts_dict(o: SolveOptsC) -> dict:
    """The scheduling fields of an options struct (as the autotuner reports them)."""
    return dict(schedule=o.schedule, group=o.group, trace_lanes=o.trace_lanes, waves_per_cu=o.waves_per_cu,
                n_bins=o.n_bins, bins_per_octave=o.bins_per_octave)


def solve(model: Model, dirset: DirSet, rays, chi, eta, freq_len, freq_dx, I_bc, origins=None, n_origins=None,
          precision: int = RT_F32, schedule: int = SCHED_DIRECT,
          waves_per_cu: int = 0, n_bins: int = 0, group: int = 0, want_u: bool = False, dtau_max: float = 0.0,
          max_substeps: int = 0, dv_max: float = 0.0, scheme: int = SCHEME_FEAUTRIER2, bins_per_octave: int = 0,
          stream=None):
    """J [n_o][F] (dtype of the precision) from ray lists; optionally u [n_o][R][F].  dtau_max > 0
    splits line intervals into optical-depth sub-steps (rt_solve_opts.dtau_max); scheme picks the
    second-order or the fourth-order Hermitian rows (rt_solve_opts.scheme)."""
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
    o = _opts(precision, schedule, waves_per_cu, n_bins, group=group, dtau_max=dtau_max,
              max_substeps=max_substeps, dv_max=dv_max, scheme=scheme, bins_per_octave=bins_per_octave)
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


def solve_noalloc(model: Model, dirset: DirSet, rays, chi, eta, freq_len, freq_dx, I_bc, J, origins=None,
                  n_origins=None, precision: int = RT_F32, schedule: int = SCHED_DIRECT, u=None, stream=None, **kw):
    """rt_solve_noalloc into the caller's J (and u, if given): the solve with the library's static
    scratch instead of a workspace.  Nothing is allocated here either: J (and u) are the caller's."""
    torch = _torch()
    dt = torch.float64 if precision == RT_F64 else torch.float32
    if origins is not None:
        origins = _dev(origins, torch.int32)
        n_origins = origins.numel()
    elif n_origins is None:
        n_origins = model.P
    ray_off, ids, Z = rays
    g, keep = _grid(freq_len, freq_dx)
    o = _opts(precision, schedule, **kw)
    _check(load().rt_solve_noalloc(model._h, dirset._h, _ptr(origins), n_origins, _ptr(ray_off), _ptr(ids), _ptr(Z),
                                   _ptr(_dev(chi, dt)), _ptr(_dev(eta, dt)), precision, chi.shape[1], C.byref(g),
                                   _ptr(_dev(I_bc, torch.float64)), _ptr(_dev(J, dt)), _ptr(u), C.byref(o),
                                   _stream(stream)))
    del keep
    return J


def compute_J_direct(model: Model, dirset: DirSet, chi, eta, freq_len, freq_dx, I_bc, origins=None, **kw):
    """J from the low-level calls: rt_trace_count + rt_trace_write over the whole list, then rt_solve."""
    rays = trace(model, dirset, origins=origins)
    return solve(model, dirset, rays, chi, eta, freq_len, freq_dx, I_bc, origins=origins, **kw)


def compute_J_workspace(dirset: DirSet, n_origins: int, F: int, precision: int = RT_F32,
                        schedule: int = SCHED_SPATIAL, mean_entries: float = 0.0) -> int:
    """Bytes with which rt_compute_J takes every origin in one chunk, for rays of mean_entries entries."""
    o = _opts(precision, schedule)
    b = _sz()
    _check(load().rt_compute_J_workspace(dirset._h, n_origins, F, C.byref(o), float(mean_entries), C.byref(b)))
    return int(b.value)


def compute_J(model: Model, dirset: DirSet, chi, eta, freq_len, freq_dx, I_bc, origins=None, n_origins=None,
              J=None, u=None, ws=None, ws_bytes: int = None, precision: int = RT_F32,
              schedule: int = SCHED_SPATIAL, want_u: bool = False, stream=None, **kw):
    """J [n_o][F] by rt_compute_J: the whole path in one library call, the origins chunked to fit the
    workspace (ws: a device uint8 tensor; default sized for one chunk at 64 entries per ray, or
    ws_bytes).  want_u also returns u [n_o][R][F]."""
    torch = _torch()
    L = load()
    dt = torch.float64 if precision == RT_F64 else torch.float32
    chi, eta = _dev(chi, dt), _dev(eta, dt)
    I_bc = _dev(I_bc, torch.float64)
    if origins is not None:
        origins = _dev(origins, torch.int32)
        n_origins = origins.numel()
    elif n_origins is None:
        n_origins = model.P
    F = int(sum(freq_len))
    R = dirset.R
    g, keep = _grid(freq_len, freq_dx)
    o = _opts(precision, schedule, **kw)
    if ws is None:
        if ws_bytes is None:
            b = _sz()
            _check(L.rt_compute_J_workspace(dirset._h, n_origins, F, C.byref(o), 0.0, C.byref(b)))
            ws_bytes = b.value
        ws = torch.empty(max(1, int(ws_bytes)), dtype=torch.uint8, device=chi.device)
    if J is None:
        J = torch.empty((n_origins, F), dtype=dt, device=chi.device)
    if want_u and u is None:
        u = torch.empty((n_origins, R, F), dtype=dt, device=chi.device)
    _check(L.rt_compute_J(model._h, dirset._h, _ptr(origins), n_origins, _ptr(chi), _ptr(eta), precision,
                          chi.shape[1], C.byref(g), _ptr(I_bc), _ptr(J), _ptr(u), C.byref(o), _ptr(ws), ws.numel(),
                          _stream(stream)))
    del keep
    return (J, u) if want_u else J


def compute_J_batched(models, dirset: DirSet, chis, etas, freq_len, freq_dx, I_bc, Js=None,
                      precision: int = RT_F32, schedule: int = SCHED_BINNED, stream=None, **kw):
    """rt_compute_J_batched: every model's J [P_k][F] from one graph over their disjoint union."""
    torch = _torch()
    dt = torch.float64 if precision == RT_F64 else torch.float32
    F = int(sum(freq_len))
    n = len(models)
    if Js is None:
        Js = [torch.empty((m.P, F), dtype=dt, device=m.pos.device) for m in models]
    chis = [_dev(c, dt) for c in chis]
    etas = [_dev(e, dt) for e in etas]
    g, keep = _grid(freq_len, freq_dx)
    o = _opts(precision, schedule, **kw)
    arr = lambda xs: (_vp * n)(*[x for x in xs])  # noqa: E731
    lds = (_i64 * n)(*[c.shape[1] for c in chis])
    _check(load().rt_compute_J_batched(n, arr([m._h.value for m in models]), dirset._h,
                                       arr([c.data_ptr() for c in chis]), arr([e.data_ptr() for e in etas]),
                                       precision, lds, C.byref(g), _ptr(_dev(I_bc, torch.float64)),
                                       arr([J.data_ptr() for J in Js]), C.byref(o), _stream(stream)))
    del keep
    return Js


class Batch:
    """Many models in one launch (rt_batch): a disjoint union built on the device, traced and solved by
    one plan, replayed as one HIP graph with the table gather and the J scatter."""

    def __init__(self, models, dirset: DirSet, chis, etas, freq_len, freq_dx, I_bc, Js, precision: int = RT_F32,
                 schedule: int = SCHED_BINNED, stream=None, **kw):
        torch = _torch()
        dt = torch.float64 if precision == RT_F64 else torch.float32
        n = len(models)
        self.models, self.dirset = list(models), dirset
        self.chis = [_dev(c, dt) for c in chis]
        self.etas = [_dev(e, dt) for e in etas]
        self.Js = [_dev(J, dt) for J in Js]
        self.I_bc = _dev(I_bc, torch.float64)
        g, self._keep = _grid(freq_len, freq_dx)
        o = _opts(precision, schedule, **kw)
        arr = lambda xs: (_vp * n)(*[x for x in xs])  # noqa: E731
        lds = (_i64 * n)(*[c.shape[1] for c in self.chis])
        h = _vp()
        _check(load().rt_batch_create(n, arr([m._h.value for m in models]), dirset._h,
                                      arr([c.data_ptr() for c in self.chis]), arr([e.data_ptr() for e in self.etas]),
                                      precision, lds, C.byref(g), _ptr(self.I_bc),
                                      arr([J.data_ptr() for J in self.Js]), C.byref(o), _stream(stream), C.byref(h)))
        self._h = h
        p = _vp()
        _check(load().rt_batch_plan(self._h, C.byref(p)))
        self._plan = p

    def union(self):
        P, E = _i64(), _i64()
        _check(load().rt_batch_union(self._h, C.byref(P), C.byref(E)))
        return P.value, E.value

    def union_index(self, stream=None):
        """Device int32 [P_total]: the union id of point i of model k at [base_k + i]
        (base_k = the points of the models before k); the inner plan's lists carry union ids."""
        torch = _torch()
        P, _ = self.union()
        idx = torch.empty(P, dtype=torch.int32, device="cuda")
        _check(load().rt_batch_union_index(self._h, idx.data_ptr(), _stream(stream)))
        return idx

    def run(self, use_graph: bool = True, stream=None):
        _check(load().rt_batch_run(self._h, 1 if use_graph else 0, _stream(stream)))

    def profile(self, n_runs: int, stream=None) -> dict:
        """Stage times (ms) of the inner plan over the union (rt_plan_profile)."""
        out = np.zeros(6)
        _check(load().rt_plan_profile(self._plan, n_runs, out.ctypes.data, _stream(stream)))
        return dict(zip(Plan.STAGES, out.tolist()))

    def info(self):
        tot = _i64()
        off, ids, Z = _vp(), _vp(), _vp()
        _check(load().rt_plan_info(self._plan, C.byref(tot), C.byref(off), C.byref(ids), C.byref(Z)))
        return dict(total=tot.value, ray_off=off.value, ray_ids=ids.value, ray_Z=Z.value)

    def rays_view(self):
        """The union's ray lists (ray_off, ids, Z; origins = every union point in order, ids union
        point ids) aliasing the inner plan's buffers (no copy; valid while the batch lives)."""
        inf = self.info()
        n = self.union()[0] * 2 * self.dirset.R + 1
        return (_view(inf["ray_off"], n, "<i8"), _view(inf["ray_ids"], inf["total"], "<i4"),
                _view(inf["ray_Z"], inf["total"], "<f8"))

    def autotune(self, n_runs: int = 2, verbose: bool = False, stream=None):
        """Tune the inner plan in place (rt_autotune_plan); returns (options dict, ms per step)."""
        best = SolveOptsC()
        ms = _dbl()
        _check(load().rt_autotune_plan(self._plan, n_runs, 1 if verbose else 0, _stream(stream), C.byref(best),
                                       C.byref(ms)))
        return opts_dict(best), ms.value

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None):
            _lib.rt_batch_destroy(self._h)
            self._h = None


def autotune(model: Model, dirset: DirSet, chi, eta, freq_len, freq_dx, I_bc, J, origins=None, n_origins=None,
             precision: int = RT_F32, n_runs: int = 2, cache_path: str = None,
             verbose: bool = False, dtau_max: float = 0.0, dv_max: float = 0.0, scheme: int = SCHEME_FEAUTRIER2,
             stream=None):
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
    base = _opts(precision, SCHED_SPATIAL, dtau_max=dtau_max, dv_max=dv_max, scheme=scheme)
    best = SolveOptsC()
    ms = _dbl()
    _check(load().rt_autotune(model._h, dirset._h, _ptr(origins), n_origins, _ptr(chi), _ptr(eta), precision,
                              chi.shape[1], C.byref(g), _ptr(I_bc), _ptr(J), C.byref(base), n_runs,
                              None if cache_path is None else cache_path.encode(), 1 if verbose else 0,
                              _stream(stream), C.byref(best), C.byref(ms)))
    del keep
    return opts_dict(best), ms.value


class Plan:
    """The whole hot path (count, scan, write, bin, sweep, reduce) as one replayable HIP graph."""

    def __init__(self, model: Model, dirset: DirSet, chi, eta, freq_len, freq_dx, I_bc, J, origins=None,
                 n_origins=None, precision: int = RT_F32, schedule: int = SCHED_DIRECT,
                 waves_per_cu: int = 0, n_bins: int = 0,
                 padded_trace_budget: int = 0, group: int = 0, trace_lanes: int = 0, walk: int = WALK_EXACT,
                 dtau_max: float = 0.0, max_substeps: int = 0, dv_max: float = 0.0,
                 scheme: int = SCHEME_FEAUTRIER2, bins_per_octave: int = 0, stream=None):
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
        o = _opts(precision, schedule, waves_per_cu, n_bins, padded_trace_budget, group, trace_lanes,
                  walk, dtau_max, max_substeps, dv_max, scheme, bins_per_octave)
        h = _vp()
        _check(load().rt_plan_create(model._h, dirset._h, _ptr(origins), n_origins, _ptr(self.chi),
                                     _ptr(self.eta), precision, self.chi.shape[1], C.byref(g), _ptr(self.I_bc),
                                     _ptr(self.J), C.byref(o), _stream(stream), C.byref(h)))
        self._h = h

    def retune(self, schedule: int = SCHED_SPATIAL, group: int = 0, trace_lanes: int = 0, waves_per_cu: int = 0,
               n_bins: int = 0, bins_per_octave: int = 0, stream=None):
        """Re-capture the plan's graph with other scheduling options."""
        o = _opts(RT_F32, schedule, waves_per_cu, n_bins, 0, group, trace_lanes, bins_per_octave=bins_per_octave)
        _check(load().rt_plan_retune(self._h, C.byref(o), _stream(stream)))

    def run(self, use_graph: bool = True, stream=None):
        _check(load().rt_plan_run(self._h, 1 if use_graph else 0, _stream(stream)))

    STAGES = ("walk", "scan", "lists", "bin", "sweep", "reduce")

    def profile(self, n_runs: int, stream=None) -> dict:
        """Mean per-stage times (ms) over n_runs eager runs, from HIP events on the stream."""
        out = np.zeros(6)
        _check(load().rt_plan_profile(self._h, n_runs, out.ctypes.data, _stream(stream)))
        return dict(zip(self.STAGES, out.tolist()))

    def copy_u(self, u=None, stream=None):
        """Per-pair mean intensities u [n_origins][R][F] of the last run (device tensor)."""
        torch = _torch()
        if u is None:
            u = torch.empty((self.n_origins, self.dirset.R, self.J.shape[1]), dtype=self.J.dtype, device=self.J.device)
        _check(load().rt_plan_copy_u(self._h, _ptr(u), _stream(stream)))
        return u

    def info(self):
        tot = _i64()
        off, ids, Z = _vp(), _vp(), _vp()
        _check(load().rt_plan_info(self._h, C.byref(tot), C.byref(off), C.byref(ids), C.byref(Z)))
        return dict(total=tot.value, ray_off=off.value, ray_ids=ids.value, ray_Z=Z.value)

    def rays_view(self):
        """The plan's own ray lists (ray_off, ids, Z) as device tensors aliasing its buffers (no
        copy; valid while the plan lives)."""
        inf = self.info()
        n = self.n_origins * 2 * self.dirset.R + 1
        return (_view(inf["ray_off"], n, "<i8"), _view(inf["ray_ids"], inf["total"], "<i4"),
                _view(inf["ray_Z"], inf["total"], "<f8"))

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


# ---------------------------------------------------------------- learned closure

MLP_D_IN = 16
MLP_NPARAM = 136450
CLOSURE_STAT_BLOCKS = 1024


class MLP:
    """The closure network (rt_mlp): FP32 master parameters, Adam state, BF16 copies on the device."""

    def __init__(self, seed: int = 0, stream=None):
        h = _vp()
        _check(load().rt_mlp_create(seed, _stream(stream), C.byref(h)))
        self._h = h
        self._ws = None

    @staticmethod
    def n_params() -> int:
        n = _i64()
        _check(load().rt_mlp_num_params(C.byref(n)))
        return n.value

    def get_params(self, stream=None) -> np.ndarray:
        out = np.empty(MLP_NPARAM, np.float32)
        _check(load().rt_mlp_get_params(self._h, out.ctypes.data, _stream(stream)))
        return out

    def set_params(self, params, stream=None):
        p = np.ascontiguousarray(params, np.float32)
        assert p.size == MLP_NPARAM
        _check(load().rt_mlp_set_params(self._h, p.ctypes.data, _stream(stream)))

    def get_grads(self, stream=None) -> np.ndarray:
        out = np.empty(MLP_NPARAM, np.float32)
        _check(load().rt_mlp_get_grads(self._h, out.ctypes.data, _stream(stream)))
        return out

    def zero_grad(self, stream=None):
        _check(load().rt_mlp_zero_grad(self._h, _stream(stream)))

    def workspace(self, n: int, device="cuda"):
        """A training workspace for up to n samples (kept by the handle)."""
        torch = _torch()
        b = _sz()
        _check(load().rt_mlp_workspace(n, 1, C.byref(b)))
        if self._ws is None or self._ws.numel() < b.value:
            self._ws = torch.empty(max(b.value, 1), dtype=torch.uint8, device=device)
        return self._ws

    def forward(self, X, n=None, rows=None, Y=None, keep=False, stream=None):
        """Y [n][2] f32 for the BF16 inputs X [*][16] (int16 bit patterns), rows optional int32 gather list."""
        torch = _torch()
        if rows is not None:
            rows = _dev(rows, torch.int32)
            n = rows.numel() if n is None else n
        elif n is None:
            n = X.shape[0]
        X = _dev(X, torch.int16)
        if Y is None:
            Y = torch.empty((n, 2), dtype=torch.float32, device=X.device)
        ws = self.workspace(n, X.device) if keep else None
        _check(load().rt_mlp_forward(self._h, _ptr(X), _ptr(rows), n, _ptr(_dev(Y, torch.float32)), 1 if keep else 0,
                                     _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream)))
        return Y

    def backward(self, X, dY, n=None, rows=None, stream=None):
        """Accumulate the gradients of sum(dY * Y) for the last keep-forward over the same samples."""
        torch = _torch()
        if rows is not None:
            rows = _dev(rows, torch.int32)
            n = rows.numel() if n is None else n
        elif n is None:
            n = X.shape[0]
        ws = self.workspace(n, X.device)
        _check(load().rt_mlp_backward(self._h, _ptr(_dev(X, torch.int16)), _ptr(rows), n,
                                      _ptr(_dev(dY, torch.float32)), _ptr(ws), ws.numel(), _stream(stream)))

    def adam_step(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, wd: float = 0.0,
                  stream=None):
        _check(load().rt_mlp_adam_step(self._h, lr, b1, b2, eps, wd, _stream(stream)))

    def train(self, X, T, n_steps: int, batch: int, total_steps: int, lr: float, lr_final: float = 0.0,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, wd: float = 0.0, seed: int = 0,
              loss_sum=None, stream=None):
        """n_steps graph-replayed training steps (rt_mlp_train) on the samples X [N][16] (BF16 bits)
        with targets T [N]; rows and the cosine learning rate follow the network's step counter."""
        torch = _torch()
        X = _dev(X, torch.int16)
        T = _dev(T, torch.float32)
        b = _sz()
        _check(load().rt_mlp_train_workspace(batch, C.byref(b)))
        if getattr(self, "_tws", None) is None or self._tws.numel() < b.value:
            self._tws = torch.empty(b.value, dtype=torch.uint8, device=X.device)
        o = TrainOptsC(batch=batch, total_steps=total_steps, lr=lr, lr_final=lr_final, b1=b1, b2=b2, eps=eps,
                       wd=wd, seed=seed)
        _check(load().rt_mlp_train(self._h, _ptr(X), _ptr(T), X.shape[0], C.byref(o), n_steps,
                                   _ptr(None if loss_sum is None else _dev(loss_sum, torch.float32)),
                                   _ptr(self._tws), self._tws.numel(), _stream(stream)))

    def set_input_norm(self, mean, inv_std):
        """The inputs' standardisation (host arrays of 16), kept by the handle for closure_J."""
        m = np.ascontiguousarray(mean, np.float32)
        s = np.ascontiguousarray(inv_std, np.float32)
        assert m.size == MLP_D_IN and s.size == MLP_D_IN
        _check(load().rt_mlp_set_input_norm(self._h, m.ctypes.data, s.ctypes.data))

    def __del__(self):
        if _lib is not None and getattr(self, "_h", None):
            _lib.rt_mlp_destroy(self._h)
            self._h = None


def mlp_nll(Y, T, rows=None, n=None, dY=None, loss_sum=None, stream=None):
    """Gaussian NLL gradient dY (and, with loss_sum, the summed loss) for targets T[rows[i]]."""
    torch = _torch()
    if rows is not None:
        rows = _dev(rows, torch.int32)
        n = rows.numel() if n is None else n
    elif n is None:
        n = Y.shape[0]
    if dY is None:
        dY = torch.empty((n, 2), dtype=torch.float32, device=Y.device)
    _check(load().rt_mlp_nll(_ptr(_dev(Y, torch.float32)), _ptr(_dev(T, torch.float32)), _ptr(rows), n,
                             _ptr(dY), _ptr(loss_sum), _stream(stream)))
    return dY


def closure_features(model: Model, chi, eta, freq_x, J1, u=None, points=None, feat=None, stream=None):
    """Features [n_points*F][16] f32 of rt_closure_features (J1 [n_points][F] f32; u optional
    [n_points][R][F] f32 per-pair coarse intensities)."""
    torch = _torch()
    chi, eta = _dev(chi, torch.float32), _dev(eta, torch.float32)
    J1 = _dev(J1, torch.float32)
    freq_x = _dev(freq_x, torch.float32)
    n_points, F = J1.shape
    R = 0
    if u is not None:
        u = _dev(u, torch.float32)
        assert u.dim() == 3 and u.shape[0] == n_points and u.shape[2] == F
        R = u.shape[1]
    if points is not None:
        points = _dev(points, torch.int32)
        assert points.numel() == n_points
    if feat is None:
        feat = torch.empty((n_points * F, MLP_D_IN), dtype=torch.float32, device=J1.device)
    _check(load().rt_closure_features(model._h, _ptr(chi), _ptr(eta), chi.shape[1], F, _ptr(freq_x), _ptr(J1),
                                      _ptr(u), R, _ptr(points), n_points, _ptr(_dev(feat, torch.float32)),
                                      _stream(stream)))
    return feat


def closure_feature_stats(feat, stream=None):
    """Column sums and sums of squares (device f64 [32]) of feat [n][16]."""
    torch = _torch()
    feat = _dev(feat, torch.float32)
    sums = torch.empty(2 * MLP_D_IN, dtype=torch.float64, device=feat.device)
    part = torch.empty(CLOSURE_STAT_BLOCKS * 2 * MLP_D_IN, dtype=torch.float64, device=feat.device)
    _check(load().rt_closure_feature_stats(_ptr(feat), feat.shape[0], _ptr(sums), _ptr(part), _stream(stream)))
    return sums


def closure_normalize(feat, mean, inv_std, X=None, stream=None):
    """BF16 (int16 bit patterns) X = (feat - mean) * inv_std; mean, inv_std host arrays of 16."""
    torch = _torch()
    feat = _dev(feat, torch.float32)
    m = np.ascontiguousarray(mean, np.float32)
    s = np.ascontiguousarray(inv_std, np.float32)
    assert m.size == MLP_D_IN and s.size == MLP_D_IN
    if X is None:
        X = torch.empty((feat.shape[0], MLP_D_IN), dtype=torch.int16, device=feat.device)
    _check(load().rt_closure_normalize(_ptr(feat), feat.shape[0], m.ctypes.data, s.ctypes.data,
                                       _ptr(_dev(X, torch.int16)), _stream(stream)))
    return X


def closure_apply(J1, Y, log_bound: float, J=None, flagged=None, n_flagged=None, stream=None):
    """J = J1 exp(m) and the fallback list; returns (J, flagged, n_flagged device int32 [1])."""
    torch = _torch()
    J1 = _dev(J1, torch.float32)
    n_points, F = J1.shape
    dev = J1.device
    if J is None:
        J = torch.empty_like(J1)
    if flagged is None:
        flagged = torch.empty(max(n_points, 1), dtype=torch.int32, device=dev)
    if n_flagged is None:
        n_flagged = torch.empty(1, dtype=torch.int32, device=dev)
    _check(load().rt_closure_apply(_ptr(J1), _ptr(_dev(Y, torch.float32)), n_points, F, float(log_bound),
                                   _ptr(_dev(J, torch.float32)), _ptr(flagged), _ptr(n_flagged), _stream(stream)))
    return J, flagged, n_flagged


def closure_merge(J_fine, flagged, n_flagged: int, J, stream=None):
    """J[flagged[k]] = J_fine[k] for k < n_flagged."""
    torch = _torch()
    J = _dev(J, torch.float32)
    _check(load().rt_closure_merge(_ptr(_dev(J_fine, torch.float32)), _ptr(_dev(flagged, torch.int32)), n_flagged,
                                   J.shape[1], J.shape[0], _ptr(J), _stream(stream)))
    return J


def closure_targets(J1, J_fine, T=None, stream=None):
    """T = log(J_fine / J1) elementwise (f32)."""
    torch = _torch()
    J1, J_fine = _dev(J1, torch.float32), _dev(J_fine, torch.float32)
    assert J1.shape == J_fine.shape
    if T is None:
        T = torch.empty(J1.numel(), dtype=torch.float32, device=J1.device)
    _check(load().rt_closure_targets(_ptr(J1), _ptr(J_fine), J1.numel(), _ptr(_dev(T, torch.float32)),
                                     _stream(stream)))
    return T


# ---------------------------------------------------------------- re-meshing indicators

# The paper's reduction parameters (Table 1): (f_small, f_large, G_thres)
REDUCTION_PARAMS = {"AMR": (0.90, 2.10, 0.10), "SPH": (1.00, 2.15, 0.21)}


def mesh_indicators(model: Model, f, f_small: float, f_large: float, G_thres: float, stream=None):
    """(Gf, L, ell) device f64 [P] for the tracer f (device f64 [P]); see rt_mesh_indicators."""
    torch = _torch()
    f = _dev(f, torch.float64)
    P = model.P
    Gf, L, ell = (torch.empty(P, dtype=torch.float64, device=f.device) for _ in range(3))
    _check(load().rt_mesh_indicators(model._h, _ptr(f), float(f_small), float(f_large), float(G_thres), _ptr(Gf),
                                     _ptr(L), _ptr(ell), _stream(stream)))
    return Gf, L, ell


def healpix_vec2pix(nside: int, dirs) -> np.ndarray:
    """Ring-scheme pixels of host directions [n][3] at resolution nside."""
    d = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    out = np.empty(len(d), np.int64)
    _check(load().rt_healpix_vec2pix(int(nside), d.ctypes.data, len(d), out.ctypes.data))
    return out


def closure_J_ws(model: Model, coarse: DirSet, F: int, solve_bytes: int):
    """A workspace for rt_closure_J (device uint8 tensor) with solve_bytes left for its solves."""
    torch = _torch()
    b = _sz()
    _check(load().rt_closure_J_workspace(model._h, coarse._h, F, int(solve_bytes), C.byref(b)))
    return torch.empty(max(1, b.value), dtype=torch.uint8, device=model.pos.device)


def closure_J(model: Model, coarse: DirSet, fine: DirSet, chi, eta, freq_len, freq_dx, freq_x0, I_bc, mlp: MLP,
              log_bound: float, solve_bytes: int, J=None, flagged=None, schedule: int = SCHED_SPATIAL, ws=None,
              stream=None):
    """rt_closure_J: the learned closure of every point in one library call; returns (J, flagged, n_flagged)."""
    torch = _torch()
    chi, eta = _dev(chi, torch.float32), _dev(eta, torch.float32)
    F = int(sum(freq_len))
    L = load()
    if ws is None:
        ws = closure_J_ws(model, coarse, F, solve_bytes)
    if J is None:
        J = torch.empty((model.P, F), dtype=torch.float32, device=chi.device)
    if flagged is None:
        flagged = torch.empty(model.P, dtype=torch.int32, device=chi.device)
    g, keep = _grid(freq_len, freq_dx, freq_x0)
    o = _opts(RT_F32, schedule)
    nf = _i64()
    _check(L.rt_closure_J(model._h, coarse._h, fine._h, _ptr(chi), _ptr(eta), chi.shape[1], C.byref(g),
                          _ptr(_dev(I_bc, torch.float64)), mlp._h, float(log_bound), _ptr(J), _ptr(flagged),
                          C.byref(nf), C.byref(o), _ptr(ws), ws.numel(), _stream(stream)))
    del keep, ws
    return J, flagged, int(nf.value)
