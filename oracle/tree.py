"""Active nodes and recursive tree evaluation of heap-ordered genotypes.

A genotype of height h has 2^(h+1)-1 slots; slot i has children 2i+1 and
2i+2 (Section 3.1: fixed-length strings mapped onto a tree template).  The
root is active; an active operator makes its first ``arity`` children active (a
unary operator reads its left child); every other slot is an intron and is
ignored (Section 3.2, Fig. 1).

The evaluation walks the tree from the root, vectorised over all rows, in
float64.  It deliberately does not use the postfix form, so it is independent
of the encoder and of the stack interpreter it is compared with.
"""
import numpy as np

from . import opset as O


def depth_of(i: int) -> int:
    return int(np.floor(np.log2(i + 1)))


def active_slots(genes_row, height: int):
    """Sorted list of the active slots of one genotype."""
    T = 2 ** (height + 1) - 1
    act = []
    todo = [0]
    while todo:
        i = todo.pop()
        if i >= T:
            raise ValueError("active node outside the template")
        act.append(i)
        g = int(genes_row[i])
        k = O.arity(g)
        if k and depth_of(i) == height:
            raise ValueError(f"active operator at leaf slot {i}")
        if not O.is_function(g) and not O.is_terminal(g):
            raise ValueError(f"active slot {i} holds no symbol ({g})")
        for c in range(k):
            todo.append(2 * i + 1 + c)
    return sorted(act)


def active_constants(genes_row, height: int):
    """Slots of the active constants, in post-order (left subtree, right
    subtree, node): the order in which a postfix program meets them."""
    out = []

    def walk(i):
        g = int(genes_row[i])
        for c in range(O.arity(g)):
            walk(2 * i + 1 + c)
        if g == O.CONST:
            out.append(i)

    walk(0)
    return out


def _chain(f, t):
    """Chain-rule product f * t with 0 * anything = 0 (see Evaluator)."""
    with np.errstate(all="ignore"):
        return np.where((f == 0) | (t == 0), 0.0, f * t)


class Evaluator:
    """Float64 tree walk over all rows of X (float64 [F, N]).

    Options
    -------
    rng       "f32": emulate binary32 overflow after every operator; "f64": none
    perturb   (rng, eps): multiply every operator result by (1 + u*eps),
              u ~ U(-1, 1) per row (Monte-Carlo arithmetic)
    record    a list; every decision input (guard / clamp / overflow) is
              appended as (array, threshold)
    thresholds (guard, clamp) of the protected operators (the defaults of
              opset; the conditioning check moves them)
    duals     if True also return d value / d constant for every active
              constant, shape [C, N], constants in post-order.  The chain
              rule's products absorb zeros: a local partial of exactly 0 (a
              guarded branch, a saturated clamp) times anything is 0, and so is
              anything times a tangent of exactly 0, even where the other
              factor is infinite (a node value that overflowed and is absorbed
              above it); elsewhere the product is the plain one
    """

    def __init__(self, X, rng="f32", perturb=None, record=None, duals=False,
                 thresholds=(O.GUARD, O.CLAMP)):
        self.X = X
        self.guard, self.clamp = thresholds
        self.N = X.shape[1]
        self.rng = rng
        self.perturb = perturb
        self.record = record
        self.duals = duals

    def run(self, genes_row, gconst_row, height: int):
        self.genes = genes_row
        self.gconst = gconst_row
        self.height = height
        self.const_slots = active_constants(genes_row, height) if self.duals else []
        self.const_index = {s: j for j, s in enumerate(self.const_slots)}
        v, d = self._ev(0)
        if self.duals and d is None:
            d = np.zeros((len(self.const_slots), self.N))
        return (v, d) if self.duals else v

    def _ev(self, i: int):
        g = int(self.genes[i])
        if g >= O.VAR0:
            v = self.X[g - O.VAR0].astype(np.float64, copy=True)
            return v, None  # a variable has no constant tangent (None = all zero)
        if g == O.CONST:
            v = np.full(self.N, float(self.gconst[i]))
            d = None
            if self.duals:
                d = np.zeros((len(self.const_slots), self.N))
                d[self.const_index[i]] = 1.0
            return v, d
        k = O.arity(g)
        if k == 0:
            raise ValueError(f"slot {i}: bad symbol {g}")
        a, da = self._ev(2 * i + 1)
        b, db = self._ev(2 * i + 2) if k == 2 else (None, None)
        v = O.apply(g, a, b, self.guard, self.clamp)
        if self.record is not None:
            self.record.extend(O.decision_inputs(g, a, b, self.guard, self.clamp))
        d = None
        if self.duals and (da is not None or db is not None):
            pa, pb = O.partials(g, a, b, v, self.guard, self.clamp)
            with np.errstate(all="ignore"):
                if da is not None:
                    d = _chain(pa[None, :], da)
                if db is not None:
                    d = _chain(pb[None, :], db) if d is None else d + _chain(pb[None, :], db)
        if self.perturb is not None:
            r, eps = self.perturb
            f = 1.0 + eps * r.uniform(-1.0, 1.0, self.N)
            v = v * f
            if d is not None:
                d = d * f[None, :]
        if self.record is not None:
            self.record.append((v, O.F32_MAX if self.rng == "f32" else np.finfo(np.float64).max))
        v = O.to_range(v, self.rng)
        return v, d


def evaluate(genes_row, gconst_row, height: int, X, rng: str = "f32"):
    """Prediction p[N] of one genotype on every row of X (float64 [F, N])."""
    return Evaluator(X, rng=rng).run(genes_row, gconst_row, height)
