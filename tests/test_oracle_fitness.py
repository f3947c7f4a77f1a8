"""Pins of Eq. 1 (MSE), Eq. 2 (NMSE) and the linear-scaling fit."""
import math

import numpy as np
import pytest

from oracle import codec, fitness as FT, opset as O, tree as TR
from synth import get_config, make_dataset

V = [O.VAR0 + k for k in range(10)]
C = O.CONST


def genotype(tokens, consts, height=6):
    ops = np.full(2 ** (height + 1) - 1, -1, dtype=np.int8)
    ops[: len(tokens)] = tokens
    cs = np.zeros(2 ** height, dtype=np.float32)
    cs[: len(consts)] = consts
    g, c = codec.decode_one(ops, cs, height)
    return g, c


def score_prog(tokens, consts, X, y, ls=True, height=6):
    g, c = genotype(tokens, consts, height)
    p = TR.evaluate(g, c, height, np.asarray(X, np.float64))
    return FT.score(p, y, ls), p


def test_eq1_mse_closed_form():
    rng = np.random.default_rng(1)
    y = rng.normal(size=500)
    d = rng.normal(size=500) * 0.1
    s = FT.score(y + d, y, linear_scaling=False)
    assert s["fitness"] == pytest.approx(np.mean(d ** 2), rel=1e-13)
    assert s["mse"] == s["fitness"]


def test_eq2_nmse_uses_population_variance():
    rng = np.random.default_rng(2)
    y = rng.normal(size=300) * 3 + 1
    p = y + 0.5
    s = FT.score(p, y, linear_scaling=False)
    assert s["nmse"] == pytest.approx(0.25 / np.var(y), rel=1e-13)  # np.var: ddof=0


def test_constant_tree():
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (2, 400))
    y = np.sin(3 * X[0]) + X[1]
    vy = np.var(y)
    s, _ = score_prog([C], [0.75], X, y, ls=True)
    assert s["fitness"] == pytest.approx(vy, rel=1e-13) and s["b"] == 0.0
    s, _ = score_prog([C], [0.75], X, y, ls=False)
    assert s["fitness"] == pytest.approx(vy + (0.75 - y.mean()) ** 2, rel=1e-13)


def test_affine_and_sign_invariance():
    rng = np.random.default_rng(4)
    X = rng.uniform(-2, 2, (3, 1000))
    y = X[0] * X[1] + np.cos(X[2])
    base = [V[0], O.SIN, V[1], O.MUL, V[2], O.ADD]          # T
    s0, _ = score_prog(base, [], X, y)
    # alpha + beta * T in a template two levels higher
    s1, _ = score_prog([C, C] + base + [O.MUL, O.ADD], [3.25, -0.4], X, y)
    # -T
    s2, _ = score_prog([C] + base + [O.SUB], [0.0], X, y)
    assert s1["fitness"] == pytest.approx(s0["fitness"], rel=1e-10)
    assert s2["fitness"] == pytest.approx(s0["fitness"], rel=1e-12)
    assert s0["fitness"] < np.var(y)


def test_two_rows_fit_exactly():
    X = np.array([[0.3, -1.2]])
    y = np.array([5.0, -7.0])
    s, _ = score_prog([V[0], O.EXP], [], X, y)
    assert s["fitness"] == pytest.approx(0.0, abs=1e-25)


def test_matches_textbook_least_squares():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(2, 777))
    y = 2 * X[0] - X[1] ** 2 + 0.3 * rng.normal(size=777)
    s, p = score_prog([V[0], V[1], O.MUL, O.SIN], [], X, y)
    A = np.stack([np.ones_like(p), p], 1)
    coef, res, *_ = np.linalg.lstsq(A, y, rcond=None)
    assert s["a"] == pytest.approx(coef[0], rel=1e-10)
    assert s["b"] == pytest.approx(coef[1], rel=1e-10)
    assert s["fitness"] == pytest.approx(res[0] / len(y), rel=1e-10)


def test_degenerate_and_nonfinite_rules():
    X = np.array([[1.0, 2.0, 3.0]])
    y = np.array([1.0, 4.0, 2.0])
    s, _ = score_prog([V[0], V[0], O.SUB, C, O.ADD], [2.0], X, y)   # constant p
    assert s["b"] == 0.0 and s["a"] == pytest.approx(y.mean()) and s["fitness"] == pytest.approx(np.var(y))
    s, _ = score_prog([V[0], C, O.MUL, C, O.MUL], [1e30, 1e10], X, y)  # 1e40 overflows f32
    assert s["status"] == 1 and s["fitness"] == math.inf


def _generating_tree_cfg2():
    # 1.5*x0*x3 - sin(x2)/(1 + x5*x5): height 4 (SUB > DIV > ADD > MUL > x5)
    return ([C, V[0], O.MUL, V[3], O.MUL, V[2], O.SIN, C, V[5], V[5], O.MUL, O.ADD, O.DIV, O.SUB],
            [1.5, 1.0])


def _generating_tree_cfg4():
    # 2.3*x0^2 - 0.7*x1*x4 + cos(1.9*x2)
    return ([C, V[0], V[0], O.MUL, O.MUL, C, V[1], O.MUL, V[4], O.MUL, O.SUB,
             C, V[2], O.MUL, O.COS, O.ADD], [2.3, 0.7, 1.9])


def test_generating_tree_fits_noise_free_target():
    cfg = get_config(4)
    X, y = make_dataset(cfg, N=20000)
    toks, cs = _generating_tree_cfg4()
    g, c = genotype(toks, cs, height=5)
    p = TR.evaluate(g, c, 5, X.astype(np.float64))
    s = FT.score(p, y)
    assert s["nmse"] <= 1e-13   # only the float32 rounding of y remains


def test_generating_tree_noisy_target_closed_form():
    cfg = get_config(2)
    N = 20000
    X, y = make_dataset(cfg, N=N)
    toks, cs = _generating_tree_cfg2()
    g, c = genotype(toks, cs, height=4)
    f = TR.evaluate(g, c, 4, X.astype(np.float64))
    s = FT.score(f, y)
    # closed form of the LS residual for y = f + e:  Var(e) - Cov(e, f)^2 / Var(f)
    e = y.astype(np.float64) - f
    cov = np.mean((e - e.mean()) * (f - f.mean()))
    want = np.var(e) - cov ** 2 / np.var(f)
    assert s["fitness"] == pytest.approx(want, rel=1e-9)
    assert s["fitness"] == pytest.approx(0.01 ** 2, rel=0.05)   # noise std 0.01
