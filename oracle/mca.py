"""Which individuals can be graded at a given node precision.

The paper notes that single-precision evaluation differs from double precision
and that some expression structures amplify the rounding (Section 5).  An
individual whose fitness is that sensitive cannot be held to a relative
tolerance close to the node precision, so it is flagged (reported, not hidden).

Monte-Carlo arithmetic (Parker, "Monte Carlo Arithmetic", 1997; cf. Vignes'
CESTAC): the individual is evaluated n more times with every operator result
multiplied by (1 + u eps), u ~ U(-1, 1) drawn per row and node, eps the unit
roundoff of the node precision (2^-24 for float32, 2^-53 for float64).  It is
flagged if
  * the spread of the fitness over the runs exceeds a tenth of the parity
    tolerance rtol*|f| + atol*Var(y), or
  * any discrete decision (a guard, a clamp, overflow, the degenerate
    linear-scaling rule, finiteness) differs between runs, or
  * any decision input lies within a relative ``window`` of its threshold.
With ``with_grad`` the gradient's normwise spread is checked the same way.
"""
import numpy as np

from . import fitness as FT
from . import grad as GR
from . import tree as TR

EPS = {"f32": 2.0 ** -24, "f64": 2.0 ** -53}
#: absolute tolerance of the parity gate, in units of Var(y)
ATOL = {"f32": 1e-10, "f64": 1e-14}


def _decisions(record):
    out = []
    with np.errstate(invalid="ignore"):
        for arr, thr in record:
            out.append(np.abs(arr) >= thr)
    return out


def _near(record, window):
    with np.errstate(invalid="ignore"):
        for arr, thr in record:
            if np.any(np.abs(np.abs(arr) - thr) <= window * thr):
                return True
    return False


def flags(genes, gconst, heights, X, y, precision="f32", rtol=1e-5, n=8, seed=0,
          linear_scaling=True, window=1e-4, with_grad=False, indices=None):
    """Boolean array (one per listed individual): True = flagged."""
    X64 = np.asarray(X, dtype=np.float64)
    y64 = np.asarray(y, dtype=np.float64)
    M = genes.shape[0]
    hs = np.broadcast_to(np.asarray(heights), (M,))
    idx = list(range(M)) if indices is None else list(indices)
    eps = EPS[precision]
    out = np.zeros(len(idx), dtype=bool)
    for q, m in enumerate(idx):
        h = int(hs[m])
        rec = []
        ev = TR.Evaluator(X64, rng=precision, record=rec, duals=with_grad)
        res = ev.run(genes[m], gconst[m], h)
        p0 = res[0] if with_grad else res
        s0 = FT.score(p0, y64, linear_scaling)
        if _near(rec, window):
            out[q] = True
            continue
        if s0["status"] == 0 and s0["vp"] <= 1e2 * FT.DEGENERATE_RTOL * max(s0["pbar"] ** 2, 1e-300) \
                and s0["vp"] > 0:
            out[q] = True
            continue
        d0 = _decisions(rec)
        g0 = GR.gradient(genes[m], gconst[m], h, X64, y64, linear_scaling, precision)[1] \
            if with_grad else None
        rs = np.random.default_rng([seed, m])
        fits, flagged = [s0["fitness"]], False
        gmax = 0.0
        for _ in range(n):
            rec_k = []
            evk = TR.Evaluator(X64, rng=precision, perturb=(rs, eps), record=rec_k, duals=with_grad)
            rk = evk.run(genes[m], gconst[m], h)
            pk = rk[0] if with_grad else rk
            sk = FT.score(pk, y64, linear_scaling)
            dk = _decisions(rec_k)
            if sk["status"] != s0["status"] or any(np.any(a != b) for a, b in zip(d0, dk)):
                flagged = True
                break
            if s0["status"] == 0 and s0["b"] == 0.0 and sk["b"] != 0.0:
                flagged = True
                break
            fits.append(sk["fitness"])
            if with_grad and s0["status"] == 0:
                dpk = rk[1]
                if linear_scaling and sk["b"] != 0.0:
                    r = sk["a"] + sk["b"] * pk - y64
                    gk = (dpk @ r) * (2.0 * sk["b"] / y64.size)
                elif not linear_scaling:
                    gk = (dpk @ (pk - y64)) * (2.0 / y64.size)
                else:
                    gk = np.zeros_like(g0)
                if g0.size:
                    gmax = max(gmax, float(np.max(np.abs(gk - g0))))
        if flagged:
            out[q] = True
            continue
        if s0["status"] == 0:
            f = np.asarray(fits)
            atol = ATOL[precision] * s0["vy"]
            if f.max() - f.min() > (rtol * abs(s0["fitness"]) + atol) / 10:
                out[q] = True
                continue
            if with_grad and g0.size:
                if gmax > (rtol * float(np.max(np.abs(g0))) + atol) / 10:
                    out[q] = True
    return out
