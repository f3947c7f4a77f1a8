"""Fitness of one prediction vector, float64.

MSE    Eq. 1:  (1/N) sum (p_i - y_i)^2
NMSE   Eq. 2:  MSE / Var(y), with the population variance (1/N), matching
               Eq. 1's 1/N (the paper does not say which variance it means)
LS-MSE linear scaling.  The paper's GPU path has none (App. A.2 says it is not
       yet supported there); this is the textbook least-squares affine fit of y
       on p, computed two-pass and centred:
           b = sum (p - pbar)(y - ybar) / sum (p - pbar)^2,  a = ybar - b pbar
       and then the direct residual pass  (1/N) sum (y - a - b p)^2.
       Degenerate case: if Var(p) <= 1e-12 * max(pbar^2, 1e-300) the fit is
       b = 0, a = ybar and LS-MSE = Var(y).
Non-finite rule: if any prediction is NaN or infinite, the fitness is +inf and
the status is 1 (a, b, MSE and NMSE are then ybar, 0, inf, inf).

Sums use math.fsum up to 2e6 terms and numpy's pairwise sum beyond.
"""
import math

import numpy as np

from . import tree as TR

DEGENERATE_RTOL = 1e-12


def _sum(v):
    v = np.asarray(v, dtype=np.float64)
    if v.size <= 2_000_000:
        return math.fsum(v.tolist()) if v.size < 20000 else float(math.fsum(v))
    return float(np.sum(v))


def target_stats(y):
    y = np.asarray(y, dtype=np.float64)
    N = y.size
    ybar = _sum(y) / N
    vy = _sum((y - ybar) ** 2) / N
    return ybar, vy


def score(p, y, linear_scaling: bool = True, degenerate_rtol: float = DEGENERATE_RTOL):
    """dict(fitness, a, b, mse, nmse, status, vp, pbar) for predictions p.
    ``degenerate_rtol`` is the threshold of the degenerate case (moved only by
    the conditioning check)."""
    p = np.asarray(p, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    N = y.size
    ybar, vy = target_stats(y)
    if not np.all(np.isfinite(p)):
        return dict(fitness=math.inf, a=ybar, b=0.0, mse=math.inf, nmse=math.inf, status=1,
                    vp=math.nan, pbar=math.nan, vy=vy, ybar=ybar)
    mse = _sum((p - y) ** 2) / N
    pbar = _sum(p) / N
    dp = p - pbar
    spp = _sum(dp * dp)
    vp = spp / N
    if vp <= degenerate_rtol * max(pbar * pbar, 1e-300):
        a, b = ybar, 0.0
        ls = vy
    else:
        b = _sum(dp * (y - ybar)) / spp
        a = ybar - b * pbar
        ls = _sum((y - a - b * p) ** 2) / N
    fit = ls if linear_scaling else mse
    nmse = fit / vy if vy > 0 else (0.0 if fit == 0 else math.inf)
    return dict(fitness=fit, a=a, b=b, mse=mse, nmse=nmse, status=0, vp=vp, pbar=pbar,
                vy=vy, ybar=ybar)


def evaluate_population(genes, gconst, heights, X, y, linear_scaling=True, rng="f32",
                        indices=None):
    """Score every (or the listed) genotype.  X float [F, N], y float [N].

    Returns dict of arrays: fitness, a, b, mse, nmse, status."""
    X64 = np.asarray(X, dtype=np.float64)
    y64 = np.asarray(y, dtype=np.float64)
    M = genes.shape[0]
    hs = np.broadcast_to(np.asarray(heights), (M,))
    idx = range(M) if indices is None else indices
    out = {k: [] for k in ("fitness", "a", "b", "mse", "nmse", "status")}
    for m in idx:
        p = TR.evaluate(genes[m], gconst[m], int(hs[m]), X64, rng=rng)
        s = score(p, y64, linear_scaling)
        for k in out:
            out[k].append(s[k])
    return {k: np.asarray(v) for k, v in out.items()}
