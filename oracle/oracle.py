"""ctypes wrapper of the C oracle (oracle.c) plus its build step.

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
CPU-baseline leg; never by the library itself.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc: FP64, no FMA contraction (fused multiply-adds only where
    written as fma), no fast-math, OpenMP."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               # call sin and cos themselves (glibc's fused sincos may differ in the last bit)
               "-fno-builtin-sin", "-fno-builtin-cos",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def build_variant(src_text: str, out_path: str) -> str:
    """Compile a modified copy of oracle.c (given as text) with the oracle's flags into out_path."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-fno-builtin-sin", "-fno-builtin-cos", "-shared", "-fPIC", "-o", out_path, src, "-lm"])
    return out_path


def load_variant(path: str):
    """A separately built oracle library, with the signature of or_compute_J_sub declared."""
    L = C.CDLL(path)
    i64, i32, vp = C.c_int64, C.c_int32, C.c_void_p
    L.or_compute_J_sub.restype = C.c_int
    L.or_compute_J_sub.argtypes = [i64, vp, vp, vp, vp, i64, i32, vp, vp, vp, vp, i64, vp, i64, vp,
                                   vp, i32, vp, i64, C.c_double, C.c_double, i64, i32, vp, vp, C.c_int]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        i64, i32, dp, vp = C.c_int64, C.c_int32, C.POINTER(C.c_double), C.c_void_p
        L.or_hp_npix.restype = i64
        L.or_hp_npix.argtypes = [i64]
        L.or_hp_pix2vec.restype = None
        L.or_hp_pix2vec.argtypes = [i64, i64, vp]
        L.or_hp_ring_of.restype = i64
        L.or_hp_ring_of.argtypes = [i64, i64]
        L.or_hp_vec2pix.restype = i64
        L.or_hp_vec2pix.argtypes = [i64, vp]
        L.or_hp_antipode.restype = i64
        L.or_hp_antipode.argtypes = [i64, i64]
        L.or_hp_parent.restype = i64
        L.or_hp_parent.argtypes = [i64, i64]
        L.or_dirset_uniform.restype = i64
        L.or_dirset_uniform.argtypes = [i64, vp, vp, vp]
        L.or_trace_ray.restype = i64
        L.or_trace_ray.argtypes = [vp, vp, vp, i64, i64, vp, vp, vp, i64]
        L.or_trace_all.restype = i64
        L.or_trace_all.argtypes = [vp, vp, vp, i64, i64, vp, i32, vp, i64, vp, vp, vp, C.c_int]
        L.or_feautrier_u.restype = C.c_double
        L.or_feautrier_u.argtypes = [i64, i64, vp, vp, C.c_double]
        L.or_feautrier_u_hermite.restype = C.c_double
        L.or_feautrier_u_hermite.argtypes = [i64, i64, vp, vp, C.c_double]
        L.or_fx_sqrt.restype = C.c_double
        L.or_fx_sqrt.argtypes = [C.c_double]
        L.or_fx_atan2.restype = C.c_double
        L.or_fx_atan2.argtypes = [C.c_double, C.c_double]
        L.or_fx_vec2pix.restype = i64
        L.or_fx_vec2pix.argtypes = [i64, vp]
        L.or_dirset_adaptive_R.restype = i64
        L.or_dirset_adaptive_R.argtypes = [i32, i32]
        L.or_dirset_adaptive.restype = i64
        L.or_dirset_adaptive.argtypes = [vp, i64, vp, i64, vp, i64, i32, i32, vp, vp, vp, vp, C.c_int]
        L.or_compute_J.restype = C.c_int
        L.or_compute_J.argtypes = [i64, vp, vp, vp, vp, i64, i32, vp, vp, vp, vp, i64, vp, i64, vp,
                                   vp, i32, vp, i64, vp, vp, C.c_int]
        L.or_compute_J_sub.restype = C.c_int
        L.or_compute_J_sub.argtypes = [i64, vp, vp, vp, vp, i64, i32, vp, vp, vp, vp, i64, vp, i64, vp,
                                       vp, i32, vp, i64, C.c_double, C.c_double, i64, i32, vp, vp, C.c_int]
        _ = dp
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ----------------------------------------------------------------- HEALPix

def hp_npix(nside: int) -> int:
    return lib().or_hp_npix(nside)


def hp_pix2vec(nside: int, p: int) -> np.ndarray:
    v = np.zeros(3)
    lib().or_hp_pix2vec(nside, p, _p(v))
    return v


def hp_ring_of(nside: int, p: int) -> int:
    return lib().or_hp_ring_of(nside, p)


def hp_vec2pix(nside: int, v) -> int:
    v = _c(v, np.float64)
    return lib().or_hp_vec2pix(nside, _p(v))


def hp_antipode(nside: int, p: int) -> int:
    return lib().or_hp_antipode(nside, p)


def hp_parent(nside: int, p: int) -> int:
    return lib().or_hp_parent(nside, p)


def dirset_uniform(nside: int):
    """(pix int64 [R], dirs float64 [R][3], w2 float64 [R]) of the uniform pair set."""
    L = lib()
    R = L.or_dirset_uniform(nside, None, None, None)
    pix = np.zeros(R, np.int64)
    dirs = np.zeros((R, 3))
    w2 = np.zeros(R)
    L.or_dirset_uniform(nside, _p(pix), _p(dirs), _p(w2))
    return pix, dirs, w2


def fx_sqrt(x: float) -> float:
    return lib().or_fx_sqrt(float(x))


def fx_atan2(y: float, x: float) -> float:
    return lib().or_fx_atan2(float(y), float(x))


def fx_vec2pix(nside: int, v) -> int:
    v = _c(v, np.float64)
    return lib().or_fx_vec2pix(nside, _p(v))


def dirset_adaptive_R(lmin: int, lmax: int) -> int:
    return lib().or_dirset_adaptive_R(lmin, lmax)


def dirset_adaptive(model, lmin: int, lmax: int, sample, origins=None, nthreads: int = 0):
    """Adaptive sets: (pix [n][R] int64, level [n][R] int32, dirs [n][R][3], w2 [n][R])."""
    L = lib()
    pos = _c(model.pos, np.float64)
    origins = np.arange(model.P, dtype=np.int32) if origins is None else _c(origins, np.int32)
    sample = _c(sample, np.int32)
    R = L.or_dirset_adaptive_R(lmin, lmax)
    n = len(origins)
    pix = np.zeros((n, R), np.int64)
    lev = np.zeros((n, R), np.int32)
    dirs = np.zeros((n, R, 3))
    w2 = np.zeros((n, R))
    L.or_dirset_adaptive(_p(pos), model.P, _p(origins), n, _p(sample), len(sample), lmin, lmax, _p(pix),
                         _p(lev), _p(dirs), _p(w2), nthreads)
    return pix, lev, dirs, w2


# ----------------------------------------------------------------- tracing

def trace_ray(model, origin: int, d) -> tuple:
    L = lib()
    d = _c(d, np.float64)
    pos = _c(model.pos, np.float64)
    off = _c(model.nbr_off, np.int64)
    idx = _c(model.nbr_idx, np.int32)
    n = L.or_trace_ray(_p(pos), _p(off), _p(idx), model.P, origin, _p(d), None, None, 0)
    ids = np.zeros(n, np.int32)
    Z = np.zeros(n)
    L.or_trace_ray(_p(pos), _p(off), _p(idx), model.P, origin, _p(d), _p(ids), _p(Z), n)
    return ids, Z


def trace_all(model, dirs, origins, nthreads: int = 0):
    """Ray lists in slot order o*2R + 2r (+n) / 2r+1 (-n). dirs [R][3] or [n_o][R][3]."""
    L = lib()
    dirs = _c(dirs, np.float64)
    per = 1 if dirs.ndim == 3 else 0
    R = dirs.shape[-2]
    origins = _c(origins, np.int32)
    pos = _c(model.pos, np.float64)
    off = _c(model.nbr_off, np.int64)
    idx = _c(model.nbr_idx, np.int32)
    n_o = len(origins)
    ray_off = np.zeros(n_o * 2 * R + 1, np.int64)
    L.or_trace_all(_p(pos), _p(off), _p(idx), model.P, R, _p(dirs), per, _p(origins), n_o,
                   _p(ray_off), None, None, nthreads)
    T = int(ray_off[-1])
    ids = np.zeros(T, np.int32)
    Z = np.zeros(T)
    L.or_trace_all(_p(pos), _p(off), _p(idx), model.P, R, _p(dirs), per, _p(origins), n_o,
                   _p(ray_off), _p(ids), _p(Z), nthreads)
    return ray_off, ids, Z


# ----------------------------------------------------------------- solve

def feautrier_u(dtau, S, m: int, I: float) -> float:
    dtau = _c(dtau, np.float64)
    S = _c(S, np.float64)
    return lib().or_feautrier_u(len(S), m, _p(dtau), _p(S), float(I))


def feautrier_u_hermite(dtau, S, m: int, I: float) -> float:
    dtau = _c(dtau, np.float64)
    S = _c(S, np.float64)
    return lib().or_feautrier_u_hermite(len(S), m, _p(dtau), _p(S), float(I))


def compute_J(model, dirs, w2, origins=None, chi=None, eta=None, I_bc=None, nthreads: int = 0,
              want_u: bool = False, dtau_max: float = 0.0, max_sub: int = 1024, dv_max: float = 0.0,
              scheme: int = 0, lib_path: str = None):
    """J[n_origins][F] (and optionally u[n_origins][R][F]) in FP64.  dv_max > 0 samples line
    intervals whose projected velocity changes by more than dv_max Doppler widths (Section 2.1.1);
    dtau_max > 0 then splits every interval into optical-depth sub-steps (Section 2.1.2, eq. 2);
    at most max_sub parts per interval for each.  scheme 0: second-order Feautrier rows; 1: the
    fourth-order Hermitian rows with third-order boundary conditions (Section 2.1).
    lib_path: another build of oracle.c to run instead (the tests check that their pins catch
    mistakes planted in a copy of the source)."""
    L = lib() if lib_path is None else load_variant(lib_path)
    dirs = _c(dirs, np.float64)
    w2 = _c(w2, np.float64)
    per = 1 if dirs.ndim == 3 else 0
    R = dirs.shape[-2]
    if origins is None:
        origins = np.arange(model.P, dtype=np.int32)
    origins = _c(origins, np.int32)
    chi = _c(model.chi if chi is None else chi, np.float64)
    eta = _c(model.eta if eta is None else eta, np.float64)
    I_bc = _c(model.I_bc if I_bc is None else I_bc, np.float64)
    pos = _c(model.pos, np.float64)
    off = _c(model.nbr_off, np.int64)
    idx = _c(model.nbr_idx, np.int32)
    vel = None if model.vel is None else _c(model.vel, np.float32)
    F = chi.shape[1]
    blk_len = _c(model.freq.len, np.int32)
    blk_dx = _c(model.freq.dx, np.float64)
    n_o = len(origins)
    J = np.zeros((n_o, F))
    u = np.zeros((n_o, R, F)) if want_u else None
    rc = L.or_compute_J_sub(model.P, _p(pos), _p(off), _p(idx), _p(vel), F, len(blk_len), _p(blk_len),
                            _p(blk_dx), _p(chi), _p(eta), chi.shape[1], _p(I_bc), R, _p(dirs), _p(w2), per,
                            _p(origins), n_o, float(dv_max), float(dtau_max), int(max_sub), int(scheme), _p(J),
                            _p(u), nthreads)
    if rc != 0:
        raise FloatingPointError("oracle produced a non-finite u (rc=%d)" % rc)
    return (J, u) if want_u else J
