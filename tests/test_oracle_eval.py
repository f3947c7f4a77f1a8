"""Pins of the oracle's tree walk: hand-computed values, identities of the
protected operators, operand order, overflow emulation."""
import json
import math
import os

import numpy as np
import pytest

from oracle import codec, opset as O, tree as TR

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig1_example.json")


def prog(tokens, consts=(), height=6):
    """Genotype of a hand-written postfix program (decoded by the oracle)."""
    ops = np.full(2 ** (height + 1) - 1, -1, dtype=np.int8)
    ops[: len(tokens)] = tokens
    cs = np.zeros(2 ** height, dtype=np.float32)
    cs[: len(consts)] = consts
    g, c = codec.decode_one(ops, cs, height)
    return g, c, height


def ev(tokens, consts, X, rng="f32"):
    g, c, h = prog(tokens, consts)
    return TR.evaluate(g, c, h, np.asarray(X, dtype=np.float64), rng=rng)


V0, V1, V2 = O.VAR0, O.VAR0 + 1, O.VAR0 + 2
C = O.CONST


def test_fig1_values():
    with open(GOLD) as f:
        g = json.load(f)
    genes = np.array(g["genes"], dtype=np.int8)
    gc = np.array(g["gene_consts"], dtype=np.float32)
    X = np.array([pt["x"] for pt in g["points"]], dtype=np.float64).T
    p = TR.evaluate(genes, gc, 3, X)
    assert p.tolist() == pytest.approx([pt["value"] for pt in g["points"]], rel=1e-15)
    assert p[1] == 1.0  # the protected branch, exactly


def test_operand_order_left_is_first():
    X = np.array([[3.0], [2.0]])
    assert ev([V0, V1, O.SUB], [], X)[0] == 1.0
    assert ev([V0, V1, O.DIV], [], X)[0] == 1.5
    assert ev([V1, V0, O.SUB], [], X)[0] == -1.0
    assert ev([V0, V1, O.POW], [], X)[0] == pytest.approx(9.0, rel=1e-15)


def test_hand_computed_small_trees():
    X = np.array([[0.5, -1.5], [2.0, 4.0]])
    # sin(x0) * x1 + 0.25
    p = ev([V0, O.SIN, V1, O.MUL, C, O.ADD], [0.25], X)
    assert p.tolist() == pytest.approx([math.sin(0.5) * 2 + 0.25, math.sin(-1.5) * 4 + 0.25], rel=1e-15)
    # exp(x0) - log(x1)
    p = ev([V0, O.EXP, V1, O.LOG, O.SUB], [], X)
    assert p.tolist() == pytest.approx([math.exp(0.5) - math.log(2), math.exp(-1.5) - math.log(4)], rel=1e-15)
    # sqrt(x1) / cos(x0) and sq(x0)
    p = ev([V1, O.SQRT, V0, O.COS, O.DIV], [], X)
    assert p.tolist() == pytest.approx([math.sqrt(2) / math.cos(0.5), 2 / math.cos(-1.5)], rel=1e-15)
    assert ev([V0, O.SQ], [], X).tolist() == [0.25, 2.25]


def test_identities():
    rng = np.random.default_rng(0)
    X = rng.uniform(-3, 3, (3, 2000))
    x0, x1 = X[0], X[1]
    # sin^2 + cos^2 = 1
    p = ev([V0, O.SIN, O.SQ, V0, O.COS, O.SQ, O.ADD], [], X)
    assert np.allclose(p, 1.0, rtol=0, atol=4e-16)
    # x0 - x0 = 0 exactly; (x0 + x1) - x1 ~ x0
    assert (ev([V0, V0, O.SUB], [], X) == 0).all()
    assert np.allclose(ev([V0, V1, O.ADD, V1, O.SUB], [], X), x0, rtol=0, atol=1e-14)
    # exp(log x) = |x| away from the guard; sqrt(sq x) = |x|; pow(x, 2) = x^2
    big = np.abs(x0) > 1e-3
    assert np.allclose(ev([V0, O.LOG, O.EXP], [], X)[big], np.abs(x0[big]), rtol=1e-14)
    assert np.allclose(ev([V0, O.SQ, O.SQRT], [], X), np.abs(x0), rtol=1e-15)
    assert np.allclose(ev([V0, C, O.POW], [2.0], X)[big], x0[big] ** 2, rtol=1e-13)
    # sqrt of a negative argument uses |a|
    assert np.allclose(ev([V0, O.SQ, C, O.MUL, O.SQRT], [-1.0], X), np.abs(x0), rtol=1e-15)


def test_guards_and_clamps():
    X = np.array([[0.3, -2.0, 0.0], [1.0, 5.0, 7.0]])
    # x0 / (x1 - x1) is always the protected value 1
    assert (ev([V0, V1, V1, O.SUB, O.DIV], [], X) == 1.0).all()
    # log(x0 - x0) = 0
    assert (ev([V0, V0, O.SUB, O.LOG], [], X) == 0.0).all()
    # pow(0, b) = 0
    assert (ev([V0, V0, O.SUB, V1, O.POW], [], X) == 0.0).all()
    # exp clamped at +-80
    p = ev([V0, C, O.MUL, O.EXP], [1000.0], X)
    assert p.tolist() == pytest.approx([math.exp(80.0), math.exp(-80.0), 1.0], rel=1e-15)
    # pow clamped: 5^(1000) -> e^80
    p = ev([V1, C, O.POW], [1000.0], X)
    assert p[1] == pytest.approx(math.exp(80.0), rel=1e-15) and p[0] == 1.0  # 1^1000 = 1
    # guard threshold is the float32 nearest to 1e-6, strict '<'
    g = float(np.float32(1e-6))
    Xg = np.array([[1.0, 1.0], [g, np.nextafter(g, 0)]])
    p = ev([V0, V1, O.DIV], [], Xg)
    assert p[0] == 1.0 / g and p[1] == 1.0


def test_nan_passes_through_clamp():
    X = np.array([[np.inf], [1.0]])
    # inf - inf = NaN; exp(clamp(NaN)) must stay NaN
    p = ev([V0, V0, O.SUB, O.EXP], [], X)
    assert np.isnan(p[0])


def test_float32_overflow_emulation():
    X = np.array([[1e30], [1e20]])
    # 1e30 * 1e20 = 1e50 overflows binary32 but not binary64
    assert np.isinf(ev([V0, V1, O.MUL], [], X, rng="f32")[0])
    assert ev([V0, V1, O.MUL], [], X, rng="f64")[0] == pytest.approx(1e50)
    # ... and the infinity is absorbed the way float32 absorbs it: a / inf = 0
    p = ev([V1, V0, V1, O.MUL, O.DIV], [], X, rng="f32")
    assert p[0] == 0.0
    # exp(clamp(inf)) = e^80, a finite value
    assert ev([V0, V1, O.MUL, O.EXP], [], X, rng="f32")[0] == pytest.approx(math.exp(80.0), rel=1e-15)
    # the rounding threshold: FLT_MAX stays finite, the next binary64 step that
    # rounds up in binary32 does not
    t = O.F32_OVERFLOW
    assert np.isinf(O.to_range(np.array([t]), "f32"))[0]
    assert np.isfinite(O.to_range(np.array([np.nextafter(t, 0)]), "f32"))[0]
    assert float(np.float32(np.nextafter(t, 0))) == O.F32_MAX
    with np.errstate(over="ignore"):
        assert np.isinf(np.float32(t))


def test_heap_walk_agrees_with_a_scalar_walk_of_the_postfix_program():
    """tree.py walks the heap-ordered genotype over all rows at once; here
    each program's postfix form (codec) is parsed and evaluated row by row
    with scalar Python arithmetic, for operators whose definition needs no
    protection.  A wrong child slot, operand order or unary operand shows."""
    from synth import Config, sample_population
    from synth import symbols as SS
    F = 4
    cfg = Config(99, "scalar-walk", 60, (3, 4, 5), (SS.ADD, SS.SUB, SS.MUL, SS.SIN, SS.COS, SS.SQ), F, 16,
                 "U", -1.5, 1.5, lambda x: x[0])
    genes, gc, hs = sample_population(cfg, M=60, salt=4)
    rng = np.random.default_rng(8)
    X = rng.uniform(-1.5, 1.5, (F, 16))
    fn = {O.ADD: lambda a, b: a + b, O.SUB: lambda a, b: a - b, O.MUL: lambda a, b: a * b,
          O.SIN: math.sin, O.COS: math.cos, O.SQ: lambda a: a * a}

    def scalar(node, row):
        s = node[0]
        if s == O.CONST:
            return node[1]
        if s >= O.VAR0:
            return float(X[s - O.VAR0, row])
        return fn[s](*[scalar(k, row) for k in node[2:]])

    for m in range(60):
        h = int(hs[m])
        syms, consts = codec.encode_one(genes[m], gc[m], h)
        tree = codec.parse(np.array(syms, dtype=np.int64), np.array(consts, dtype=np.float32))
        want = [scalar(tree, r) for r in range(16)]
        got = TR.evaluate(genes[m], gc[m], h, X)
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)
