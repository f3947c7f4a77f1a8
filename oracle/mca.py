"""How sensitive each individual's fitness and gradient are to the node
precision: the tolerance the parity gate gives it.

The paper notes that single-precision evaluation differs from double precision
and that some expression structures amplify the rounding (Section 5).  So an
individual is graded with a tolerance that includes its own measured
sensitivity, rather than excluded.

Monte-Carlo arithmetic (Parker, "Monte Carlo Arithmetic", 1997; cf. Vignes'
CESTAC): the individual is evaluated n more times with every operator result
multiplied by (1 + u eps), u ~ U(-1, 1) drawn per row and node, eps the unit
roundoff of the node precision (2^-24 for float32, 2^-53 for float64).  Two more
evaluations move the discrete decisions' thresholds instead: the protection
guard and the clamp by a relative `window` (one run each way: more guarded and
less clamped, then the opposite) and the degenerate-fit threshold of linear
scaling by a factor 100 (up, then down), so that a decision whose input sits
within the window of its threshold is taken both ways.

Per individual, ``sensitivity`` reports
  * fit_spread: the largest |f_k - f_0| over those n + 2 runs (inf if a run's
    status differs from the unperturbed one: then either status is possible);
  * grad_spread: the same for the gradient in the max norm (with_grad);
  * a_spread, b_spread: the same for the linear-scaling intercept and slope;
  * flipped: a discrete decision (guard, clamp, overflow, degenerate fit,
    finiteness) differed between runs;
  * near: a decision input lies within `window` (relative) of its threshold.
``flags`` keeps the older yes/no reading: flagged if flipped, near, or a
spread exceeds a tenth of the gate rtol |v| + atol Var(y).
"""
import numpy as np

from . import fitness as FT
from . import grad as GR
from . import opset as O
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


def _gradient(dp, p, s, y64, linear_scaling):
    """Gradient of the fitness from forward-mode tangents dp [C, N] (as in
    grad.gradient, summed with a matrix product: a perturbed run needs no
    exact sum)."""
    if s["status"] != 0:
        return np.zeros(dp.shape[0])
    if linear_scaling:
        if s["b"] == 0.0:
            return np.zeros(dp.shape[0])
        return (dp @ (s["a"] + s["b"] * p - y64)) * (2.0 * s["b"] / y64.size)
    return (dp @ (p - y64)) * (2.0 / y64.size)


def sensitivity(genes, gconst, heights, X, y, precision="f32", n=8, seed=0,
                linear_scaling=True, window=1e-4, with_grad=False, indices=None):
    """One dict per listed individual: fitness, status, fit_spread,
    grad_spread (None without with_grad), flipped, near."""
    X64 = np.asarray(X, dtype=np.float64)
    y64 = np.asarray(y, dtype=np.float64)
    M = genes.shape[0]
    hs = np.broadcast_to(np.asarray(heights), (M,))
    idx = list(range(M)) if indices is None else list(indices)
    eps = EPS[precision]
    out = []
    for m in idx:
        h = int(hs[m])
        rec = []
        ev = TR.Evaluator(X64, rng=precision, record=rec, duals=with_grad)
        res = ev.run(genes[m], gconst[m], h)
        p0 = res[0] if with_grad else res
        s0 = FT.score(p0, y64, linear_scaling)
        g0 = GR.gradient(genes[m], gconst[m], h, X64, y64, linear_scaling, precision)[1] \
            if with_grad else None
        d0 = _decisions(rec)
        info = dict(fitness=s0["fitness"], status=s0["status"], fit_spread=0.0,
                    grad_spread=0.0 if with_grad else None, a_spread=0.0, b_spread=0.0,
                    flipped=False, near=_near(rec, window))
        if s0["status"] == 0 and s0["vp"] <= 1e2 * FT.DEGENERATE_RTOL * max(s0["pbar"] ** 2, 1e-300) \
                and s0["vp"] > 0:
            info["near"] = True
        rs = np.random.default_rng([seed, m])
        runs = [("mca", None)] * n + [("shift", +1), ("shift", -1)]
        for kind, sgn in runs:
            rec_k = []
            if kind == "mca":
                evk = TR.Evaluator(X64, rng=precision, perturb=(rs, eps), record=rec_k, duals=with_grad)
                drt = FT.DEGENERATE_RTOL
            else:
                thr = (O.GUARD * (1 + sgn * window), O.CLAMP * (1 - sgn * window))
                evk = TR.Evaluator(X64, rng=precision, record=rec_k, duals=with_grad, thresholds=thr)
                drt = FT.DEGENERATE_RTOL * (1e2 if sgn > 0 else 1e-2)
            rk = evk.run(genes[m], gconst[m], h)
            pk = rk[0] if with_grad else rk
            sk = FT.score(pk, y64, linear_scaling, degenerate_rtol=drt)
            if sk["status"] != s0["status"]:
                info["flipped"] = True
                info["fit_spread"] = info["a_spread"] = info["b_spread"] = np.inf
                if with_grad:
                    info["grad_spread"] = np.inf
                continue
            if any(np.any(a != b) for a, b in zip(d0, _decisions(rec_k))):
                info["flipped"] = True
            if s0["status"] == 0 and (s0["b"] == 0.0) != (sk["b"] == 0.0):
                info["flipped"] = True
            if s0["status"] != 0:
                continue
            info["fit_spread"] = max(info["fit_spread"], abs(sk["fitness"] - s0["fitness"]))
            info["a_spread"] = max(info["a_spread"], abs(sk["a"] - s0["a"]))
            info["b_spread"] = max(info["b_spread"], abs(sk["b"] - s0["b"]))
            if with_grad and g0.size:
                gk = _gradient(rk[1], pk, sk, y64, linear_scaling)
                info["grad_spread"] = max(info["grad_spread"], float(np.max(np.abs(gk - g0))))
        out.append(info)
    return out


def flags(genes, gconst, heights, X, y, precision="f32", rtol=1e-5, n=8, seed=0,
          linear_scaling=True, window=1e-4, with_grad=False, indices=None):
    """Boolean array (one per listed individual): True = flagged
    (ill-conditioned for the node precision)."""
    M = genes.shape[0]
    idx = list(range(M)) if indices is None else list(indices)
    sens = sensitivity(genes, gconst, heights, X, y, precision, n, seed, linear_scaling, window,
                       with_grad, idx)
    vy = float(np.var(np.asarray(y, dtype=np.float64)))
    out = np.zeros(len(idx), dtype=bool)
    for q, (m, s) in enumerate(zip(idx, sens)):
        if s["flipped"] or s["near"]:
            out[q] = True
            continue
        if s["status"] != 0:
            continue
        atol = ATOL[precision] * vy
        if s["fit_spread"] > (rtol * abs(s["fitness"]) + atol) / 10:
            out[q] = True
            continue
        if with_grad and s["grad_spread"]:
            g0 = GR.gradient(genes[m], gconst[m], int(np.broadcast_to(np.asarray(heights), (M,))[m]),
                             X, y, linear_scaling, precision)[1]
            if g0.size and s["grad_spread"] > (rtol * float(np.max(np.abs(g0))) + atol) / 10:
                out[q] = True
    return out
