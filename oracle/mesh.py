"""Re-meshing indicators of Section 2.2.2, written out per point.

TEST INFRASTRUCTURE ONLY (used by tests).  Plain numpy; no code shared with
the HIP library.

For a tracer f on the points of a mesh with neighbour lists:
    Gf_i  = max over neighbours n of |(f_i - f_n) / (f_i + f_n)|     (eq. 6)
    L_i   = mean over neighbours n of |x_i - x_n|                     (eq. 8)
    ell_i = L_i * f_small  if Gf_i >= G_thres,  else L_i * f_large    (eq. 7)
with the paper's parameters (Table 1): AMR (0.90, 2.10, 0.10), SPH (1.00, 2.15, 0.21).
"""
from __future__ import annotations

import numpy as np

TABLE1 = {"AMR": (0.90, 2.10, 0.10), "SPH": (1.00, 2.15, 0.21)}


def mesh_indicators(model, f, f_small, f_large, G_thres):
    off, idx, pos = model.nbr_off, model.nbr_idx, model.pos
    P = len(off) - 1
    f = np.asarray(f, np.float64)
    Gf = np.zeros(P)
    L = np.zeros(P)
    for i in range(P):
        nb = idx[off[i]:off[i + 1]]
        Gf[i] = np.max(np.abs((f[i] - f[nb]) / (f[i] + f[nb])))
        d = pos[nb] - pos[i]
        L[i] = np.mean(np.sqrt(np.sum(d * d, axis=1)))
    ell = L * np.where(Gf >= G_thres, f_small, f_large)
    return Gf, L, ell
