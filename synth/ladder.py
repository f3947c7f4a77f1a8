"""The generating expressions of the formula-ladder workloads (Tab. 1), laid on
template genotypes: a test input, not part of any evaluation.

An expression is a nested tuple: ("x", k) for variable k, or (op, left,
right) / (op, child) with op a symbol code of synth.symbols.  ``genotype``
places it at the root of a heap-ordered template of the given height (children
of slot i at 2i+1 and 2i+2); every slot the expression does not use is an
intron and holds a seeded random symbol, so the generating tree also exercises
the encoder's intron skipping.
"""
import numpy as np

from . import symbols as S
from .population import template_size


def _x(k):
    return ("x", k)


def _sum(ks):
    """Balanced sum of the variables ks."""
    if len(ks) == 1:
        return _x(ks[0])
    h = (len(ks) + 1) // 2
    return (S.ADD, _sum(ks[:h]), _sum(ks[h:]))


def _diffs(square):
    """(x4 - x3) + (x6 - x5) + (x8 - x7), each difference squared if asked."""
    parts = [(S.SUB, _x(a), _x(b)) for a, b in ((4, 3), (6, 5), (8, 7))]
    if square:
        parts = [(S.SQ, p) for p in parts]
    return (S.ADD, (S.ADD, parts[0], parts[1]), parts[2])


_PROD012 = (S.MUL, (S.MUL, _x(0), _x(1)), _x(2))

#: workload id -> generating expression (Tab. 1, Experiment III rows)
GENERATING = {
    6: _sum(list(range(9))),
    7: (S.DIV, _sum([0, 1, 2]), _sum([3, 4, 5, 6, 7, 8])),
    8: (S.DIV, _sum([0, 1, 2]), _diffs(False)),
    9: (S.DIV, _PROD012, _diffs(False)),
    10: (S.DIV, _PROD012, _diffs(True)),
}


def height_of(e) -> int:
    if e[0] == "x":
        return 0
    return 1 + max(height_of(c) for c in e[1:])


def genotype(e, height, F, funcs, seed=0):
    """(genes int8 [T], gene_consts float32 [T]) of a height-``height``
    template whose active tree is ``e``; introns drawn from ``seed``."""
    T = template_size(height)
    if height_of(e) > height:
        raise ValueError(f"expression of height {height_of(e)} does not fit height {height}")
    rng = np.random.default_rng([seed, 4242])
    depth = np.floor(np.log2(np.arange(T) + 1)).astype(np.int64)
    intr_f = np.asarray(funcs, dtype=np.int64)[rng.integers(0, len(funcs), T)]
    intr_t = np.where(rng.random(T) < 0.5, S.CONST, S.VAR0 + rng.integers(0, F, T))
    genes = np.where(depth < height, intr_f, intr_t).astype(np.int8)
    gconst = np.where(genes == S.CONST, rng.uniform(-1, 1, T), 0.0).astype(np.float32)

    def place(node, slot):
        if node[0] == "x":
            genes[slot] = S.VAR0 + node[1]
            gconst[slot] = 0.0
            return
        genes[slot] = node[0]
        for q, child in enumerate(node[1:]):
            place(child, 2 * slot + 1 + q)

    place(e, 0)
    return genes, gconst
