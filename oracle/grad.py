"""Gradient of the fitness with respect to an individual's constants, float64.

Forward mode: the tree walk carries, next to every node value, its partial
derivatives with respect to each active constant (dual numbers; one tangent row
per constant, constants in the postfix order of appearance).  Operator
partials are those of ``opset.partials`` (a guard or saturated clamp has
derivative 0).

Linear-scaling fitness: LS-MSE(c) = min over (a, b) of (1/N) sum (y - a - b p)^2.
At the optimum the partial derivatives in a and b vanish, so (envelope
theorem) d LS-MSE / d c_j = (2b/N) sum_r (a + b p_r - y_r) d p_r / d c_j, with
(a, b) the fit of ``fitness.score``.  In the degenerate case b = 0 the
gradient is 0.  Raw MSE: d MSE / d c_j = (2/N) sum_r (p_r - y_r) d p_r / d c_j.
Non-finite individuals get a zero gradient (status 1).

``gradient`` also returns, in the score dict, ``gabs[j]`` = (2|b|/N) sum_r
|(a + b p_r - y_r) d p_r / d c_j| (or the raw-MSE analogue): the sum of the
magnitudes of the terms of the gradient's dot product, which bounds the
rounding error of any evaluation of it (the standard dot-product error bound
|fl(sum t_r) - sum t_r| <= gamma sum |t_r| with gamma a small multiple of the
unit roundoff; Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1).

``fd_gradient`` is an independent check by central finite differences of the
whole fitness in float64.
"""
import numpy as np

from . import fitness as FT
from . import tree as TR


def gradient(genes_row, gconst_row, height, X, y, linear_scaling=True, rng="f32"):
    """(score dict, grad[C]) for one genotype; C = number of active constants."""
    X64 = np.asarray(X, dtype=np.float64)
    y64 = np.asarray(y, dtype=np.float64)
    ev = TR.Evaluator(X64, rng=rng, duals=True)
    p, dp = ev.run(genes_row, gconst_row, height)
    s = FT.score(p, y64, linear_scaling)
    C = dp.shape[0]
    N = y64.size
    s["gabs"] = np.zeros(C)
    if s["status"] != 0:
        return s, np.zeros(C)
    if linear_scaling:
        if s["b"] == 0.0:
            return s, np.zeros(C)
        r = s["a"] + s["b"] * p - y64
        scale = 2.0 * s["b"] / N
    else:
        r = p - y64
        scale = 2.0 / N
    g = np.array([FT._sum(r * dp[j]) for j in range(C)]) * scale
    s["gabs"] = np.array([FT._sum(np.abs(r * dp[j])) for j in range(C)]) * abs(scale)
    return s, g


def _fitness_with(genes_row, gconst_row, height, X64, y64, slot, value, linear_scaling, rng):
    gc = np.array(gconst_row, dtype=np.float64)
    gc[slot] = value
    p = TR.Evaluator(X64, rng=rng).run(genes_row, gc, height)
    return FT.score(p, y64, linear_scaling)["fitness"]


def fd_gradient(genes_row, gconst_row, height, X, y, h=1e-4, linear_scaling=True, rng="f64"):
    """Central differences (f(c+h) - f(c-h)) / 2h for every active constant,
    perturbing the float64 constant (not rounded to float32)."""
    X64 = np.asarray(X, dtype=np.float64)
    y64 = np.asarray(y, dtype=np.float64)
    slots = TR.active_constants(genes_row, height)
    g = np.zeros(len(slots))
    base = np.asarray(gconst_row, dtype=np.float64)
    for j, s in enumerate(slots):
        fp = _fitness_with(genes_row, base, height, X64, y64, s, base[s] + h, linear_scaling, rng)
        fm = _fitness_with(genes_row, base, height, X64, y64, s, base[s] - h, linear_scaling, rng)
        g[j] = (fp - fm) / (2.0 * h)
    return g
