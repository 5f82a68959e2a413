"""Learned closure driver: coarse solve, features, network, fallback.

Every arithmetic step runs in the library's kernels: the solves are one
rt_compute_J call each, inference with its fallback is one rt_closure_J call,
and training steps call rt_mlp_* (forward, loss, backward, Adam).  This module
owns the device buffers, draws the minibatch indices and builds the training
set and its standardisation.

Closure (an addition to the method, which computes J from the direction set
alone): J at nside = 1 (6 pairs, Section 2.1.3) plus local optical properties
are mapped to the J of the nside = 8 set (384 pairs).  The network predicts
m = log(J8/J1) and s, the log variance of that prediction; a point whose
predicted standard deviation exp(s/2) exceeds the bound for some frequency is
re-solved at nside = 8 (the fallback) and merged back.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import binding as rt

COARSE_NSIDE = 1
FINE_NSIDE = 8


def _torch():
    import torch
    return torch


class DeviceModel:
    """One model resident on the device: mesh handle, FP32 tables, frequency grid."""

    def __init__(self, pos, nbr_off, nbr_idx, vel, chi, eta, freq_len, freq_dx, freq_x, I_bc, name="model"):
        torch = _torch()
        self.name = name
        self.P, self.F = chi.shape
        self.model = rt.Model.from_numpy(pos, nbr_off, nbr_idx, vel)
        dev = "cuda"
        self.chi = torch.as_tensor(np.ascontiguousarray(chi, np.float32), device=dev)
        self.eta = torch.as_tensor(np.ascontiguousarray(eta, np.float32), device=dev)
        self.freq_len = list(freq_len)
        self.freq_dx = list(freq_dx)
        self.freq_x0 = None
        self.x = torch.as_tensor(np.ascontiguousarray(freq_x, np.float32), device=dev)
        self.I_bc = torch.as_tensor(np.ascontiguousarray(I_bc, np.float64), device=dev)

    @classmethod
    def from_synth(cls, m):
        dm = cls(m.pos, m.nbr_off, m.nbr_idx, m.vel, m.chi, m.eta, m.freq.len, m.freq.dx, m.freq.x(), m.I_bc,
                 name=f"{m.name}{m.meta.get('seed', '')}")
        dm.freq_x0 = list(m.freq.x0)
        return dm


@dataclass
class SolveResult:
    J: object
    ms: float                  # HIP-event time of the rt_compute_J call
    u: object = None           # per-pair mean intensities [n][R][F] when asked for


# Room for ray lists (and the per-chunk parts) that solve_J gives rt_compute_J; the library
# cuts the origins into chunks that fit it.
SOLVE_WS_BYTES = 24 << 30


def solve_J(dm: DeviceModel, dirset: "rt.DirSet", origins=None, J=None, schedule: int = rt.SCHED_SPATIAL,
            keep_u: bool = False, ws_bytes: int = SOLVE_WS_BYTES, verbose: bool = False) -> SolveResult:
    """J [n][F] (f32) for the listed origins (device int32, or all points) by one rt_compute_J call,
    which takes the origins in Morton-ordered chunks that fit ws_bytes; keep_u also returns the
    per-pair u."""
    torch = _torch()
    n = dm.P if origins is None else int(origins.numel())
    if J is None:
        J = torch.empty((max(n, 1), dm.F), dtype=torch.float32, device="cuda")[:n]
    U = torch.empty((max(n, 1), dirset.R, dm.F), dtype=torch.float32, device="cuda")[:n] if keep_u else None
    if n == 0:
        return SolveResult(J, 0.0, U)
    need = rt.compute_J_workspace(dirset, n, dm.F, schedule=schedule)
    ws = torch.empty(min(need, ws_bytes), dtype=torch.uint8, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    rt.compute_J(dm.model, dirset, dm.chi, dm.eta, dm.freq_len, dm.freq_dx, dm.I_bc, origins=origins,
                 n_origins=n, J=J, u=U, ws=ws, schedule=schedule, want_u=keep_u)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    del ws
    rt.sync_status()
    if verbose:
        print(f"  [{dm.name}] nside-{int(round(math.sqrt(dirset.R / 6)))} solve of {n} origins: {ms:.0f} ms",
              flush=True)
    return SolveResult(J, ms, U)


@dataclass
class Normalizer:
    mean: np.ndarray
    inv_std: np.ndarray

    @classmethod
    def from_sums(cls, sums: np.ndarray, n: int) -> "Normalizer":
        mean = sums[:16] / n
        var = np.maximum(sums[16:] / n - mean * mean, 0.0)
        inv = np.where(var > 1e-12 * np.maximum(1.0, mean * mean), 1.0 / np.sqrt(np.maximum(var, 1e-300)), 0.0)
        return cls(mean.astype(np.float32), inv.astype(np.float32))


def features(dm: DeviceModel, J1, u=None, points=None):
    return rt.closure_features(dm.model, dm.chi, dm.eta, dm.x, J1, u=u, points=points)


@dataclass
class ClosureNet:
    mlp: "rt.MLP"
    norm: Normalizer
    history: List[float] = field(default_factory=list)


def train(X, T, norm: Normalizer, steps: int = 20000, batch: int = 8192, lr: float = 1e-3,
          lr_final: float = 1e-5, wd: float = 0.0, seed: int = 0, log_every: int = 2000,
          verbose: bool = True) -> ClosureNet:
    """Adam on the mean Gaussian NLL over minibatches drawn with replacement from the samples X
    (BF16 bits, [N][16]) with targets T ([N]), cosine learning-rate decay: rt_mlp_train, one
    captured step replayed log_every times per call (rows drawn on the device from the seed)."""
    torch = _torch()
    net = rt.MLP(seed=seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    t0 = time.time()
    done = 0
    while done < steps:
        k = min(log_every, steps - done)
        net.train(X, T, k, batch=batch, total_steps=steps, lr=lr, lr_final=lr_final, wd=wd, seed=seed,
                  loss_sum=loss)
        done += k
        avg = loss.item() / (k * batch)
        loss.zero_()
        hist.append(avg)
        if verbose:
            a = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * (done - 1) / max(1, steps)))
            print(f"  train step {done}/{steps}: mean NLL {avg:.4f}, lr {a:.2e}, {time.time() - t0:.1f} s",
                  flush=True)
    torch.cuda.synchronize()
    net.set_input_norm(norm.mean, norm.inv_std)
    return ClosureNet(net, norm, hist)


@dataclass
class ClosureResult:
    J: object
    n_flagged: int
    total_ms: float            # HIP-event time of the rt_closure_J call (coarse solve to merge)
    flagged: object = None     # device int32, the first n_flagged entries are the flagged points


def infer(net: ClosureNet, dm: DeviceModel, coarse_set: "rt.DirSet", fine_set: "rt.DirSet", log_bound: float,
          ws_bytes: int = SOLVE_WS_BYTES) -> ClosureResult:
    """Closure J for every point of dm by one rt_closure_J call: coarse solve, features, network,
    flags, the fine solve of the flagged points and the merge all run in the library."""
    torch = _torch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    solve_bytes = min(rt.compute_J_workspace(fine_set, dm.P, dm.F), ws_bytes)
    ws = rt.closure_J_ws(dm.model, coarse_set, dm.F, solve_bytes)
    e0.record()
    J, flagged, n_flag = rt.closure_J(dm.model, coarse_set, fine_set, dm.chi, dm.eta, dm.freq_len, dm.freq_dx,
                                      dm.freq_x0, dm.I_bc, net.mlp, log_bound, solve_bytes, ws=ws)
    e1.record()
    e1.synchronize()
    rt.sync_status()
    return ClosureResult(J, n_flag, e0.elapsed_time(e1), flagged)


def rel_errors(J, J_ref) -> np.ndarray:
    """|J - J_ref| / J_ref per (point, f), on the host (float64)."""
    a = J.double().cpu().numpy()
    b = J_ref.double().cpu().numpy()
    return (np.abs(a - b) / np.abs(b)).ravel()


def flagged_mask(flagged, n_flagged: int, P: int) -> np.ndarray:
    mask = np.zeros(P, bool)
    mask[flagged[:n_flagged].cpu().numpy()] = True
    return mask


def error_summary(J, J_ref, flagged_mask: Optional[np.ndarray], F: int) -> dict:
    e = rel_errors(J, J_ref)
    out = dict(median=float(np.median(e)), p99=float(np.quantile(e, 0.99)), max=float(e.max()))
    if flagged_mask is not None:
        keep = np.repeat(~flagged_mask, F)
        ek = e[keep]
        out.update(median_unflagged=float(np.median(ek)) if ek.size else 0.0,
                   p99_unflagged=float(np.quantile(ek, 0.99)) if ek.size else 0.0,
                   flagged_fraction=float(flagged_mask.mean()))
    return out


# ---------------------------------------------------------------- experiment: train on some models, test on others

@dataclass
class Labelled:
    dm: DeviceModel
    coarse: SolveResult    # nside 1
    fine: SolveResult      # nside 8 (the label, and the plain method the closure is compared with)


def label(dm: DeviceModel, coarse_set, fine_set, verbose: bool = False) -> Labelled:
    c = solve_J(dm, coarse_set, keep_u=True, verbose=verbose)
    f = solve_J(dm, fine_set, verbose=verbose)
    return Labelled(dm, c, f)


def dataset(labelled: List[Labelled]):
    """Normalised BF16 inputs X [N][16], targets T [N] = log(J8/J1) and the normaliser, over all samples."""
    torch = _torch()
    feats = [features(lab.dm, lab.coarse.J, lab.coarse.u) for lab in labelled]
    n = sum(f.shape[0] for f in feats)
    sums = np.zeros(32)
    for f in feats:
        sums += rt.closure_feature_stats(f).cpu().numpy()
    norm = Normalizer.from_sums(sums, n)
    X = torch.empty((n, 16), dtype=torch.int16, device="cuda")
    T = torch.empty(n, dtype=torch.float32, device="cuda")
    o = 0
    for f, lab in zip(feats, labelled):
        k = f.shape[0]
        rt.closure_normalize(f, norm.mean, norm.inv_std, X=X[o:o + k])
        rt.closure_targets(lab.coarse.J, lab.fine.J, T=T[o:o + k])
        o += k
    del feats
    torch.cuda.synchronize()
    return X, T, norm


def predicted_sd(net: ClosureNet, dm: DeviceModel, coarse: SolveResult) -> np.ndarray:
    """Per point, the largest predicted standard deviation exp(s/2) over its frequencies (host)."""
    X = rt.closure_normalize(features(dm, coarse.J, coarse.u), net.norm.mean, net.norm.inv_std)
    Y = net.mlp.forward(X)
    s = Y[:, 1].reshape(dm.P, dm.F).max(1).values
    return np.exp(0.5 * s.double().cpu().numpy())


def evaluate(net: ClosureNet, lab: Labelled, coarse_set, fine_set, flag_fractions=(0.0,), mid_set=None,
             verbose: bool = False) -> dict:
    """Closure against the plain nside-8 solve on one model.  For each target fallback fraction q
    the bound is the (1 - q) quantile of the predicted per-point deviation (q = 0: no fallback;
    q = 1: every point).  Baselines: J1 alone, and J at mid_set's nside."""
    dm = lab.dm
    F = dm.F
    out = dict(model=dm.name, points=dm.P, F=F, plain_ms=lab.fine.ms, coarse_ms=lab.coarse.ms,
               coarse_alone=error_summary(lab.coarse.J, lab.fine.J, None, F))
    if mid_set is not None:
        mid = solve_J(dm, mid_set)
        out["mid_alone"] = dict(error_summary(mid.J, lab.fine.J, None, F), ms=mid.ms,
                                nside=int(round(math.sqrt(mid_set.R / 6))))
        del mid
    sd = predicted_sd(net, dm, lab.coarse)
    out["predicted_sd_quantiles"] = {str(q): float(np.quantile(sd, q)) for q in (0.1, 0.25, 0.5, 0.75, 0.9)}
    runs = []
    e_net = None  # per (point, frequency) errors of the network alone (no fallback)
    for q in flag_fractions:
        if q <= 0:
            b = math.inf
        elif q >= 1:
            b = 0.0
        else:
            b = float(np.quantile(sd, 1.0 - q))
        lb = math.log(b) if b > 0 else -math.inf
        res = infer(net, dm, coarse_set, fine_set, lb)
        mask = flagged_mask(res.flagged, res.n_flagged, dm.P)
        e = error_summary(res.J, lab.fine.J, mask, F)
        e.update(target_fraction=q, bound=b, n_flagged=res.n_flagged, total_ms=res.total_ms,
                 speedup_vs_plain=lab.fine.ms / res.total_ms if res.total_ms > 0 else None)
        if res.n_flagged == 0 and e_net is None:
            e_net = rel_errors(res.J, lab.fine.J).reshape(dm.P, F)
        runs.append(e)
        if verbose:
            print(f"  [{dm.name}] fallback {e['flagged_fraction']:.3f} (bound {b:.3g}): median "
                  f"{e['median']:.2e} (unflagged {e['median_unflagged']:.2e}), closure {res.total_ms:.0f} ms "
                  f"vs plain {lab.fine.ms:.0f} ms", flush=True)
        del res
    out["closure"] = runs
    if e_net is not None:
        if verbose:
            print(f"  [{dm.name}] fallback fraction for the target median ...", flush=True)
        out["fallback_for_target"] = fallback_curve(e_net, sd, runs, lab.fine.ms)
    return out


def fallback_curve(e_net, sd, runs, plain_ms, target: float = 1e-3) -> dict:
    """The smallest fallback fraction at which the median relative error over every (point,
    frequency) reaches `target`.  A fallen-back point carries the plain fine solve's J exactly
    (error 0, bit for bit), the others the network's, and points fall back in decreasing order
    of predicted deviation, so the median at fraction q follows from the network-only errors
    and the predictions without running the fallback at every q.  The time at that fraction is
    interpolated linearly between the measured closure runs."""
    P, F = e_net.shape
    order = np.argsort(-sd, kind="stable")
    qs = np.linspace(0.0, 1.0, 201)
    med = {}

    def median_at(i):  # the median over every (point, frequency) with the first round(q_i P) points fallen back
        if i not in med:
            e = e_net.copy()
            e[order[:int(round(qs[i] * P))]] = 0.0
            med[i] = float(np.median(e))
        return med[i]

    # A fallen-back entry becomes 0, at or below every error, so no order statistic rises with q and
    # the median is non-increasing along the grid: the first grid point reaching the target is found
    # by bisection instead of evaluating all 201 (each median runs over P F values).
    hit = None
    if median_at(len(qs) - 1) <= target:
        lo, hi = 0, len(qs) - 1
        while lo < hi:
            mid = (lo + hi) // 2
            if median_at(mid) <= target:
                hi = mid
            else:
                lo = mid + 1
        hit = lo
    q_star = float(qs[hit]) if hit is not None else None
    med_unflagged = None
    if hit is not None:
        rest = e_net[order[int(round(qs[hit] * P)):]]
        med_unflagged = float(np.median(rest)) if rest.size else 0.0
    pts = sorted((r["flagged_fraction"], r["total_ms"]) for r in runs)
    t_star = float(np.interp(q_star, [p for p, _ in pts], [t for _, t in pts])) if q_star is not None else None
    return dict(target=target, fraction=q_star, median_unflagged_at_fraction=med_unflagged,
                closure_ms_interpolated=t_star, plain_ms=plain_ms,
                speedup_vs_plain=plain_ms / t_star if t_star else None,
                curve={f"{qs[i]:.2f}": median_at(i) for i in range(0, len(qs), 10)})
