"""Pins of the oracle's constant gradient: analytic values, the linear-scaling
invariances, each operator partial against finite differences, and the whole
gradient against central finite differences."""
import numpy as np
import pytest

from oracle import codec, grad as GR, opset as O, tree as TR
from synth import get_config, make_dataset, sample_population

C = O.CONST
V0, V1, V2 = O.VAR0, O.VAR0 + 1, O.VAR0 + 2


def genotype(tokens, consts, height=5):
    ops = np.full(2 ** (height + 1) - 1, -1, dtype=np.int8)
    ops[: len(tokens)] = tokens
    cs = np.zeros(2 ** height, dtype=np.float32)
    cs[: len(consts)] = consts
    return codec.decode_one(ops, cs, height)


def test_raw_mse_analytic():
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (1, 500))
    y = 3 * X[0]
    c = 1.75
    g, gc = genotype([C, V0, O.MUL], [c])
    s, gr = GR.gradient(g, gc, 5, X, y, linear_scaling=False, rng="f64")
    assert gr[0] == pytest.approx(2 * (c - 3) * np.mean(X[0] ** 2), rel=1e-13)


def test_ls_scale_and_offset_constants_have_zero_gradient():
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (2, 800))
    y = np.sin(2 * X[0]) + X[1] ** 2
    # alpha + beta * sin(c * x0 + x1): alpha, beta are absorbed by the fit
    toks = [C, C, C, V0, O.MUL, V1, O.ADD, O.SIN, O.MUL, O.ADD]
    g, gc = genotype(toks, [0.3, 1.7, 1.4])
    s, gr = GR.gradient(g, gc, 5, X, y, rng="f64")
    assert abs(gr[0]) < 1e-14 and abs(gr[1]) < 1e-14 * max(1, abs(gr[2]))
    assert abs(gr[2]) > 1e-3


def test_gradient_term_magnitudes():
    """gabs of p = c * x0 with raw MSE is (2/N) sum |(c x - y) x|, written out;
    and |g| <= gabs always (triangle inequality)."""
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (1, 300))
    y = 0.5 * X[0] + rng.normal(0, 0.1, 300)
    c = 1.25
    g, gc = genotype([C, V0, O.MUL], [c])
    s, gr = GR.gradient(g, gc, 5, X, y, linear_scaling=False, rng="f64")
    want = 2.0 / 300 * sum(abs((c * X[0, r] - y[r]) * X[0, r]) for r in range(300))
    assert s["gabs"][0] == pytest.approx(want, rel=1e-13)
    assert abs(gr[0]) <= s["gabs"][0]
    toks = [C, C, C, V0, O.MUL, V1, O.ADD, O.SIN, O.MUL, O.ADD]
    X2 = rng.uniform(-1, 1, (2, 400))
    g2, gc2 = genotype(toks, [0.3, 1.7, 1.4])
    s2, gr2 = GR.gradient(g2, gc2, 5, X2, X2[0] ** 2, rng="f64")
    assert np.all(np.abs(gr2) <= s2["gabs"] * (1 + 1e-12))
    assert s2["gabs"][0] > 1e3 * abs(gr2[0])   # the absorbed offset cancels


@pytest.mark.parametrize("op", range(11))
def test_each_operator_partial(op):
    """d op / d a (and d b) against central differences of opset.apply."""
    rng = np.random.default_rng(op)
    a = rng.uniform(0.2, 2.5, 200) * rng.choice([-1, 1], 200)
    b = rng.uniform(0.2, 2.5, 200) * rng.choice([-1, 1], 200)
    if op == O.POW:
        a = np.abs(a)
    h = 1e-6
    v = O.apply(op, a, b)
    pa, pb = O.partials(op, a, b, v)
    fa = (O.apply(op, a + h, b) - O.apply(op, a - h, b)) / (2 * h)
    assert np.allclose(pa, fa, rtol=1e-6, atol=1e-8)
    if O.arity(op) == 2:
        fb = (O.apply(op, a, b + h) - O.apply(op, a, b - h)) / (2 * h)
        assert np.allclose(pb, fb, rtol=1e-6, atol=1e-8)


def test_guarded_branches_have_zero_partials():
    z = np.array([0.0, 5e-7])
    one = np.ones(2)
    assert (O.partials(O.DIV, one, z, O.apply(O.DIV, one, z))[0] == 0).all()
    assert (O.partials(O.LOG, z, None, O.apply(O.LOG, z))[0] == 0).all()
    big = np.array([81.0, -90.0])
    assert (O.partials(O.EXP, big, None, O.apply(O.EXP, big))[0] == 0).all()
    assert (O.partials(O.SQRT, np.zeros(1), None, np.zeros(1))[0] == 0).all()


def test_forward_mode_matches_central_fd_on_population():
    cfg = get_config(4)
    X, y = make_dataset(cfg, N=3000)
    genes, gc, hs = sample_population(cfg, M=40, salt=7)
    checked = 0
    for m in range(len(genes)):
        s, gr = GR.gradient(genes[m], gc[m], 5, X, y, rng="f64")
        if s["status"] != 0 or gr.size == 0:
            continue
        f1 = GR.fd_gradient(genes[m], gc[m], 5, X, y, h=1e-4)
        f2 = GR.fd_gradient(genes[m], gc[m], 5, X, y, h=5e-5)
        tol = 1e-6 * np.max(np.abs(f1)) + 1e-12 * s["vy"]
        if np.max(np.abs(f1 - f2)) > tol:    # kink (guard / clamp) nearby
            continue
        assert np.max(np.abs(gr - f1)) <= tol, m
        checked += 1
    assert checked >= 20


def test_zero_partial_absorbs_an_overflowed_factor():
    """q = x2 / (exp(c x0) * (x1 * x1)) with x1 * x1 beyond the binary32
    range: the denominator is infinite in the range emulation and q = 0 on
    every row, whatever c is.  Along the way, the partial of the product
    with respect to exp(c x0) is x1 * x1 = inf while exp's tangent is exactly
    0 (c x0 is beyond the clamp).  The derivative is 0 (central differences
    of the constant q = 0), not the NaN of a plain inf * 0."""
    N = 64
    X = np.stack([np.full(N, 100.0), np.full(N, 1e20), np.ones(N)])
    y = np.random.default_rng(3).standard_normal(N)
    toks = [V2, C, V0, O.MUL, O.EXP, V1, V1, O.MUL, O.MUL, O.DIV]
    g, gc = genotype(toks, [1.0])
    s, gr = GR.gradient(g, gc, 5, X, y, linear_scaling=False, rng="f32")
    p = TR.evaluate(g, gc, 5, X, rng="f32")
    assert np.all(p == 0.0) and s["status"] == 0
    fd = GR.fd_gradient(g, gc, 5, X, y, h=1e-4, linear_scaling=False, rng="f32")
    assert np.array_equal(fd, [0.0])
    assert np.array_equal(gr, [0.0]), gr
    # and the product rule itself: 0 * inf and inf * 0 give 0, finite factors multiply
    assert np.array_equal(TR._chain(np.array([0.0, np.inf, 2.0]), np.array([np.inf, 0.0, 3.0])),
                          [0.0, 0.0, 6.0])
