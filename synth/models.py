"""Seeded synthetic models shaped like the paper's workloads.

The paper's own models (an analytic Archimedean-spiral wind meshed with Gmsh,
AMR-octree and SPH snapshots of spiral outflows; Section 3) are not available,
so every model here is synthetic: a point cloud with Delaunay (or octree
adjacency) neighbour lists, which is all the method needs (Section 2.2: a point
cloud plus nearest-neighbour information), per-point opacity chi[p][f] and
emissivity eta[p][f] on per-block uniform comoving frequency grids, per-point
velocities in Doppler widths, and a boundary intensity per frequency.

Conventions shared by every consumer:
  pos      float64 [P][3]
  nbr_off  int64   [P+1]   CSR offsets
  nbr_idx  int32   [E]     neighbour ids, ascending within each row, no self
  vel      float32 [P][3]  Doppler widths (None for a static model)
  chi, eta float64 [P][F]  row-major, frequency contiguous
  freq     FreqGrid: blocks of len[b] points, x = x0[b] + j*dx[b]
  I_bc     float64 [F]
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.spatial as sps


@dataclass
class FreqGrid:
    len: np.ndarray  # int32 [B]
    x0: np.ndarray   # float64 [B]
    dx: np.ndarray   # float64 [B]

    @property
    def F(self) -> int:
        return int(self.len.sum())

    def x(self) -> np.ndarray:
        return np.concatenate([self.x0[b] + self.dx[b] * np.arange(self.len[b])
                               for b in range(len(self.len))])

    @staticmethod
    def uniform(blocks: int, n: int, lo: float = -5.0, hi: float = 5.0) -> "FreqGrid":
        dx = (hi - lo) / (n - 1) if n > 1 else 1.0
        return FreqGrid(np.full(blocks, n, np.int32), np.full(blocks, lo, np.float64),
                        np.full(blocks, dx, np.float64))


@dataclass
class Model:
    name: str
    pos: np.ndarray
    nbr_off: np.ndarray
    nbr_idx: np.ndarray
    vel: Optional[np.ndarray]
    chi: np.ndarray
    eta: np.ndarray
    freq: FreqGrid
    I_bc: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def P(self) -> int:
        return self.pos.shape[0]

    @property
    def E(self) -> int:
        return int(self.nbr_idx.shape[0])

    @property
    def F(self) -> int:
        return self.chi.shape[1]


# ----------------------------------------------------------------------------- neighbour lists

def csr_from_edges(P: int, a: np.ndarray, b: np.ndarray):
    """Symmetric, de-duplicated, self-free CSR from an undirected edge list."""
    a = np.asarray(a, np.int64)
    b = np.asarray(b, np.int64)
    keep = a != b
    a, b = a[keep], b[keep]
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    key = np.unique(src * P + dst)
    src = key // P
    dst = key % P
    off = np.zeros(P + 1, np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off)
    return off, dst.astype(np.int32)


def delaunay_csr(pos: np.ndarray):
    """Neighbour lists = edges of the Delaunay tetrahedralisation (Section 2.2)."""
    tri = sps.Delaunay(pos)
    s = tri.simplices.astype(np.int64)
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    a = np.concatenate([s[:, i] for i, _ in pairs])
    b = np.concatenate([s[:, j] for _, j in pairs])
    off, idx = csr_from_edges(pos.shape[0], a, b)
    if np.any(np.diff(off) == 0):
        raise ValueError("Delaunay left a point without neighbours")
    return off, idx


def gaussian_profile(x: np.ndarray) -> np.ndarray:
    """Unit-peak Gaussian line profile in Doppler-width units."""
    return np.exp(-x * x)


def to_fp32_tables(chi: np.ndarray, eta: np.ndarray):
    """Round the tables to float32 and return (chi32, eta32, chi64_of_32, eta64_of_32).

    The float64 copies hold exactly the float32 values, so an FP64 reference
    and an FP32 kernel see identical inputs.
    """
    c32 = np.ascontiguousarray(chi, np.float32)
    e32 = np.ascontiguousarray(eta, np.float32)
    return c32, e32, c32.astype(np.float64), e32.astype(np.float64)


# ----------------------------------------------------------------------------- models

def sphere_model(seed: int = 1, n_inner: int = 999, n_surf: int = 200, F: int = 31,
                 chi0: float = 2.0, S0: float = 1.0, I_bc: float = 0.0) -> Model:
    """Homogeneous unit sphere: an explicit centre point, n_inner uniform points in
    the ball and n_surf uniform points on the sphere; constant chi and S."""
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n_inner, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    r = rng.uniform(0.0, 1.0, n_inner) ** (1.0 / 3.0)
    inner = u * r[:, None]
    s = rng.normal(size=(n_surf, 3))
    s /= np.linalg.norm(s, axis=1)[:, None]
    pos = np.concatenate([np.zeros((1, 3)), inner, s]).astype(np.float64)
    off, idx = delaunay_csr(pos)
    P = pos.shape[0]
    freq = FreqGrid.uniform(1, F)
    chi = np.full((P, F), chi0, np.float64)
    eta = chi * S0
    return Model("sphere", pos, off, idx, None, chi, eta, freq, np.full(F, I_bc, np.float64),
                 meta=dict(seed=seed, chi0=chi0, S0=S0, I_bc=I_bc, R=1.0, centre=0))


def wind_model(seed: int = 2, P: int = 50_000, F: int = 64, r_in: float = 1.0, r_out: float = 100.0,
               chi0: float = 10.0, v_inf: float = 20.0, floor: float = 1e-4, moving: bool = True) -> Model:
    """Analytic spherical wind.

    Point density proportional to r^-3 (local element size proportional to r),
    so the radius is log-uniform on [r_in, r_out] and the direction isotropic.
    rho = r^-2, chi = chi0*rho*(phi(x) + floor), S = 1/r, eta = chi*S, radial
    velocity v(r) = v_inf*(1 - 1/r)^(1/2) Doppler widths.
    """
    rng = np.random.default_rng(seed)
    r = np.exp(rng.uniform(np.log(r_in), np.log(r_out), P))
    u = rng.normal(size=(P, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    pos = (u * r[:, None]).astype(np.float64)
    off, idx = delaunay_csr(pos)
    freq = FreqGrid.uniform(1, F)
    x = freq.x()
    rho = r ** -2.0
    chi = chi0 * rho[:, None] * (gaussian_profile(x)[None, :] + floor)
    S = 1.0 / r
    eta = chi * S[:, None]
    vel = None
    if moving:
        vr = v_inf * np.sqrt(1.0 - r_in / r)
        vel = (u * vr[:, None]).astype(np.float32)
    return Model("wind", pos, off, idx, vel, chi, eta, freq, np.zeros(F), meta=dict(seed=seed, r=r))


def tiny_model(seed: int, P: int = 40, F: int = 8, moving: bool = False) -> Model:
    """A small random Delaunay mesh in the unit cube with random positive tables."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-1.0, 1.0, (P, 3))
    off, idx = delaunay_csr(pos)
    freq = FreqGrid.uniform(1, F)
    chi = rng.uniform(0.2, 3.0, (P, F))
    eta = chi * rng.uniform(0.1, 2.0, (P, F))
    vel = rng.normal(0.0, 1.5, (P, 3)).astype(np.float32) if moving else None
    return Model("tiny", pos, off, idx, vel, chi, eta, freq, rng.uniform(0.0, 0.5, F),
                 meta=dict(seed=seed))


def lattice_model(n: int = 6, F: int = 4, spacing: float = 1.0) -> Model:
    """Cubic n^3 lattice with face (6-neighbour) connectivity."""
    g = np.arange(n)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1).astype(np.float64) * spacing
    lin = np.arange(n ** 3).reshape(n, n, n)
    a, b = [], []
    for ax in range(3):
        sl0 = [slice(None)] * 3
        sl1 = [slice(None)] * 3
        sl0[ax] = slice(0, n - 1)
        sl1[ax] = slice(1, n)
        a.append(lin[tuple(sl0)].ravel())
        b.append(lin[tuple(sl1)].ravel())
    off, idx = csr_from_edges(n ** 3, np.concatenate(a), np.concatenate(b))
    freq = FreqGrid.uniform(1, F)
    P = n ** 3
    chi = np.ones((P, F))
    eta = np.ones((P, F))
    return Model("lattice", pos, off, idx, None, chi, eta, freq, np.zeros(F), meta=dict(n=n))


# ----------------------------------------------------------------------------- AMR-octree-like cloud

def _grf(n: int, rng: np.random.Generator, slope: float = -11.0 / 3.0) -> np.ndarray:
    """Periodic Gaussian random field on n^3 with power spectrum k^slope, unit variance."""
    k = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n
    K2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kz[None, None, :] ** 2
    K2[0, 0, 0] = 1.0
    amp = K2 ** (slope / 4.0)
    amp[0, 0, 0] = 0.0
    wn = rng.normal(size=(n, n, n))
    f = np.fft.irfftn(np.fft.rfftn(wn) * amp, s=(n, n, n), axes=(0, 1, 2))
    f -= f.mean()
    f /= f.std()
    return f


def _block_minmax(a: np.ndarray, s: int):
    n = a.shape[0] // s
    b = a.reshape(n, s, n, s, n, s)
    return b.max(axis=(1, 3, 5)), b.min(axis=(1, 3, 5))


def _octree_leaves(logrho: np.ndarray, lmin: int, lmax: int, thr: float):
    """Leaves (level, i, j, k) of an octree refined where max-min of log rho in a cell > thr."""
    nfine = logrho.shape[0]
    assert nfine == 2 ** lmax
    leaves = []
    active = np.ones((2 ** lmin,) * 3, bool)
    for L in range(lmin, lmax + 1):
        if L == lmax:
            refine = np.zeros_like(active)
        else:
            mx, mn = _block_minmax(logrho, nfine >> L)
            refine = active & ((mx - mn) > thr)
        leaf = active & ~refine
        ijk = np.argwhere(leaf)
        leaves.append(np.concatenate([np.full((len(ijk), 1), L), ijk], 1))
        if L < lmax:
            active = np.repeat(np.repeat(np.repeat(refine, 2, 0), 2, 1), 2, 2)
    return np.concatenate(leaves).astype(np.int64)


def _octree_adjacency(leaves: np.ndarray, lmax: int):
    """Neighbours = leaves that touch (share a face, an edge or a corner)."""
    nf = 2 ** lmax
    P = len(leaves)
    owner = np.empty((nf, nf, nf), np.int32)
    size = nf >> leaves[:, 0]
    lo = leaves[:, 1:] * size[:, None]
    for s in np.unique(size):
        sel = np.nonzero(size == s)[0]
        for dx in range(s):
            for dy in range(s):
                for dz in range(s):
                    owner[lo[sel, 0] + dx, lo[sel, 1] + dy, lo[sel, 2] + dz] = sel
    src, dst = [], []
    for s in np.unique(size):
        sel = np.nonzero(size == s)[0]
        rng_ = np.arange(-1, s + 1)
        sh = np.array([(a, b, c) for a in rng_ for b in rng_ for c in rng_
                       if a in (-1, s) or b in (-1, s) or c in (-1, s)])
        for chunk in np.array_split(sel, max(1, len(sel) * len(sh) // 4_000_000 + 1)):
            q = lo[chunk][:, None, :] + sh[None, :, :]
            ok = np.all((q >= 0) & (q < nf), axis=2)
            qi = owner[np.clip(q[..., 0], 0, nf - 1), np.clip(q[..., 1], 0, nf - 1),
                       np.clip(q[..., 2], 0, nf - 1)]
            a = np.broadcast_to(chunk[:, None], qi.shape)[ok]
            src.append(a)
            dst.append(qi[ok])
    return csr_from_edges(P, np.concatenate(src), np.concatenate(dst))


def octree_model(seed: int = 3, lmin: int = 5, lmax: int = 8, target: int = 500_000,
                 nblocks: int = 2, nf_block: int = 48, chi0: float = 100.0, v_rms: float = 3.0,
                 floor: float = 1e-4) -> Model:
    """AMR-octree-like cloud: log-normal density from a k^(-11/3) Gaussian random field,
    octree-refined from level lmin to lmax by the spread of log rho inside a cell, the
    threshold bisected to give about `target` leaves.  Points are leaf centres in the
    unit box; neighbours are touching leaves; velocities are three further random
    fields scaled to v_rms Doppler widths; line b has strength chi0/(b+1)."""
    rng = np.random.default_rng(seed)
    n = 2 ** lmax
    g = _grf(n, rng)
    logrho = g - 0.5
    lo_t, hi_t = 0.0, float(logrho.max() - logrho.min())
    leaves = None
    for _ in range(40):
        mid = 0.5 * (lo_t + hi_t)
        lv = _octree_leaves(logrho, lmin, lmax, mid)
        if leaves is None or abs(len(lv) - target) < abs(len(leaves) - target):
            leaves = lv
        if abs(len(lv) - target) <= 0.02 * target:
            break
        if len(lv) > target:
            lo_t = mid
        else:
            hi_t = mid
    off, idx = _octree_adjacency(leaves, lmax)
    size = (n >> leaves[:, 0]).astype(np.float64)
    cen_vox = leaves[:, 1:] * size[:, None] + 0.5 * size[:, None]
    pos = (cen_vox / n).astype(np.float64)
    ci = np.clip(np.floor(cen_vox).astype(np.int64), 0, n - 1)
    rho = np.exp(logrho[ci[:, 0], ci[:, 1], ci[:, 2]])
    vel = np.stack([_grf(n, rng)[ci[:, 0], ci[:, 1], ci[:, 2]] for _ in range(3)], 1)
    vel *= v_rms / np.sqrt((vel ** 2).sum(1).mean())
    freq = FreqGrid.uniform(nblocks, nf_block)
    xb = freq.x()[:nf_block]
    prof = np.concatenate([gaussian_profile(xb) / (b + 1) for b in range(nblocks)])
    chi = chi0 * rho[:, None] * (prof[None, :] + floor)
    S = rho ** 0.3
    eta = chi * S[:, None]
    return Model("octree", pos, off, idx, vel.astype(np.float32), chi, eta, freq,
                 np.zeros(freq.F), meta=dict(seed=seed, levels=leaves[:, 0]))


# ----------------------------------------------------------------------------- SPH-like clouds

def sph_cloud_model(seed: int, P: int, F: int = 64, chi0: float = 1.0, v0: float = 10.0,
                    floor: float = 1e-4) -> Model:
    """SPH-like particle cloud: 80% Plummer sphere (a = 1, truncated at 10a) and 20% a
    logarithmic spiral arm r = exp(b*theta), b = tan 15 deg, theta in [0, 4 pi], in a
    Gaussian tube; Keplerian rotation about z.  The density used for chi and S is the
    analytic sampling density (Plummer plus tube), not a mesh estimate."""
    rng = np.random.default_rng(seed)
    n_pl = int(round(0.8 * P))
    n_arm = P - n_pl
    # Plummer: r = a / sqrt(m^(-2/3) - 1) with the mass fraction m truncated at r = 10a.
    m_max = (10.0 ** 3) / (1.0 + 10.0 ** 2) ** 1.5
    m = rng.uniform(1e-6, m_max, n_pl)
    r = 1.0 / np.sqrt(m ** (-2.0 / 3.0) - 1.0)
    u = rng.normal(size=(n_pl, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    p_pl = u * r[:, None]
    b = np.tan(np.deg2rad(15.0))
    th = rng.uniform(0.0, 4.0 * np.pi, n_arm)
    ra = np.exp(b * th) * 0.5
    centre = np.stack([ra * np.cos(th), ra * np.sin(th), np.zeros(n_arm)], 1)
    p_arm = centre + rng.normal(size=(n_arm, 3)) * np.stack([0.1 * ra, 0.1 * ra, 0.05 * ra], 1)
    pos = np.concatenate([p_pl, p_arm]).astype(np.float64)
    off, idx = delaunay_csr(pos)
    rr = np.linalg.norm(pos, axis=1)
    rho = 0.8 * (1.0 + rr ** 2) ** -2.5 + 0.2 * np.exp(-0.5 * (pos[:, 2] / (0.05 + 0.05 * rr)) ** 2) / (1.0 + rr ** 2)
    rho = rho / rho.max() * 100.0
    freq = FreqGrid.uniform(1, F)
    chi = chi0 * rho[:, None] * (gaussian_profile(freq.x())[None, :] + floor)
    S = rho ** 0.3
    eta = chi * S[:, None]
    Rc = np.maximum(np.hypot(pos[:, 0], pos[:, 1]), 0.1)
    vphi = v0 * Rc ** -0.5
    vel = np.stack([-vphi * pos[:, 1] / Rc, vphi * pos[:, 0] / Rc, np.zeros(P)], 1)
    return Model("sph", pos, off, idx, vel.astype(np.float32), chi, eta, freq, np.zeros(F),
                 meta=dict(seed=seed))


def _sph_one(args):
    seed, P, F = args
    return sph_cloud_model(seed, P, F=F)


def sph_batch_models(n_models: int = 64, seed0: int = 400, lo: int = 10_000, hi: int = 200_000,
                     F: int = 64, scale: float = 1.0, workers: int = 0) -> List[Model]:
    """n_models independent SPH-like clouds with log-uniform sizes in [lo, hi] (times scale).
    workers > 1 builds the clouds in that many processes (same result)."""
    jobs = []
    for k in range(n_models):
        rng = np.random.default_rng(seed0 + k)
        P = int(np.exp(rng.uniform(np.log(lo), np.log(hi))) * scale)
        jobs.append((seed0 + k, max(P, 64), F))
    if workers and workers > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(_sph_one, jobs))
    return [_sph_one(j) for j in jobs]


def concat_models(models: List[Model], spacing: float = 100.0) -> Model:
    """Disjoint union of models with the same frequency grid: neighbour ids are
    offset so no ray crosses from one model into another, and model k is
    translated to cell k of a cubic grid of the given spacing so the models also
    occupy disjoint regions of space.  meta["offsets"] gives each model's first
    point."""
    n = len(models)
    side = int(np.ceil(n ** (1.0 / 3.0)))
    pos, off, idx, vel, chi, eta = [], [np.zeros(1, np.int64)], [], [], [], []
    base_p, base_e, starts = 0, 0, []
    for k, m in enumerate(models):
        cell = np.array([k % side, (k // side) % side, k // (side * side)], np.float64)
        pos.append(m.pos + spacing * cell)
        off.append(m.nbr_off[1:] + base_e)
        idx.append(m.nbr_idx.astype(np.int64) + base_p)
        vel.append(m.vel if m.vel is not None else np.zeros((m.P, 3), np.float32))
        chi.append(m.chi)
        eta.append(m.eta)
        starts.append(base_p)
        base_p += m.P
        base_e += m.E
    return Model("batch", np.concatenate(pos), np.concatenate(off), np.concatenate(idx).astype(np.int32),
                 np.concatenate(vel).astype(np.float32), np.concatenate(chi), np.concatenate(eta), models[0].freq,
                 models[0].I_bc.copy(), meta=dict(offsets=np.array(starts + [base_p]), n_models=n))
