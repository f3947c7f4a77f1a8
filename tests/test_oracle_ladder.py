"""Pins of the formula-ladder workloads (Tab. 1, Experiment III) on the oracle.

The generating expression of each workload, laid on a depth-6 and a depth-8
template with random introns, must reproduce its target: NMSE (Eq. 2) far
below the paper's success threshold of 1e-6 (only the binary32 rounding of y
remains).  Two mutations tie the pin to the structure the paper discusses for
these problems: swapping the operands of one subtraction breaks Subtraction
(a non-commutative operator; no affine map of the output repairs it), while
the same swap under a square leaves Squaring exact, since (a - b)^2 = (b - a)^2.
"""
import numpy as np
import pytest

from oracle import codec, fitness as FT, tree as TR
from synth import LADDER, get_config, ladder, make_dataset
from synth import symbols as S

N = 20000


def _nmse(e, cid, height, ls=True):
    cfg = get_config(cid)
    X, y = make_dataset(cfg, N=N)
    g, c = ladder.genotype(e, height, cfg.F, cfg.funcs, seed=cid + height)
    p = TR.evaluate(g, c, height, X.astype(np.float64))
    return FT.score(p, y, ls)


@pytest.mark.parametrize("height", [6, 8])
@pytest.mark.parametrize("cid", sorted(LADDER))
def test_generating_tree_recovers_the_target(cid, height):
    e = ladder.GENERATING[cid]
    assert ladder.height_of(e) <= 6
    for ls in (True, False):
        s = _nmse(e, cid, height, ls)
        assert s["status"] == 0
        assert s["nmse"] <= 1e-12, (cid, height, ls, s["nmse"])


def test_generating_tree_is_the_active_tree():
    """The encoder keeps exactly the expression's nodes (introns dropped)."""
    cfg = get_config(10)
    g, c = ladder.genotype(ladder.GENERATING[10], 8, cfg.F, cfg.funcs, seed=1)
    syms, consts = codec.encode_one(g, c, 8)
    # x0 x1 * x2 * | 3 x (x x - sq) | 2 x + | /  ->  5 + 12 + 2 + 1 = 20 tokens
    assert len(syms) == 20 and consts == []
    assert syms[:5] == [S.VAR0, S.VAR0 + 1, S.MUL, S.VAR0 + 2, S.MUL] and syms[-1] == S.DIV


def _swap_first_sub(e):
    """The expression with the operands of its first subtraction swapped."""
    done = [False]

    def walk(n):
        if n[0] == "x":
            return n
        if n[0] == S.SUB and not done[0]:
            done[0] = True
            return (S.SUB, n[2], n[1])
        return (n[0],) + tuple(walk(k) for k in n[1:])

    out = walk(e)
    assert done[0]
    return out


def test_subtraction_order_matters():
    s = _nmse(_swap_first_sub(ladder.GENERATING[8]), 8, 6)
    assert s["nmse"] > 1e-3


def test_squaring_makes_subtraction_order_irrelevant():
    s = _nmse(_swap_first_sub(ladder.GENERATING[10]), 10, 6)
    assert s["nmse"] <= 1e-12


def test_denominators_are_kept_away_from_zero():
    for cid in (8, 9, 10):
        cfg = get_config(cid)
        X, y = make_dataset(cfg, N=N)
        assert np.all(np.abs(cfg.den(X.astype(np.float64))) >= 0.01)
        assert np.all(np.isfinite(y))
