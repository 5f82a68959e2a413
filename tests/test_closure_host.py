"""Host logic of the closure driver: the fallback fraction that reaches a target median."""
import numpy as np
import pytest

from paper_2011_14998_amd import closure as cl


def _scan(e_net, sd, target):
    """Every grid fraction evaluated, in order: the definition the bisection must reproduce."""
    P = e_net.shape[0]
    order = np.argsort(-sd, kind="stable")
    qs = np.linspace(0.0, 1.0, 201)
    med, unfl = [], []
    for q in qs:
        k = int(round(q * P))
        e = e_net.copy()
        e[order[:k]] = 0.0
        med.append(float(np.median(e)))
        rest = e_net[order[k:]]
        unfl.append(float(np.median(rest)) if rest.size else 0.0)
    hit = np.nonzero(np.array(med) <= target)[0]
    return qs, med, unfl, (int(hit[0]) if hit.size else None)


@pytest.mark.parametrize("P,F,target,seed", [(500, 8, 1e-3, 1), (333, 5, 2e-2, 2), (64, 3, 0.5, 3), (257, 4, 0.0, 4)])
def test_fallback_curve_matches_full_scan(P, F, target, seed):
    rng = np.random.default_rng(seed)
    e_net = np.abs(rng.lognormal(-3.0, 1.5, (P, F)))
    e_net[rng.random((P, F)) < 0.05] = 0.0          # some exact zeros
    sd = np.round(rng.random(P), 2)                 # ties in the predicted deviation
    runs = [dict(flagged_fraction=0.0, total_ms=1.0), dict(flagged_fraction=1.0, total_ms=9.0)]
    got = cl.fallback_curve(e_net, sd, runs, plain_ms=10.0, target=target)
    qs, med, unfl, hit = _scan(e_net, sd, target)
    assert got["fraction"] == (float(qs[hit]) if hit is not None else None)
    assert got["median_unflagged_at_fraction"] == (unfl[hit] if hit is not None else None)
    assert got["curve"] == {f"{q:.2f}": m for q, m in zip(qs[::10], med[::10])}
