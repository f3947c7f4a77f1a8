"""The conditioning flags separate well- from ill-conditioned individuals."""
import numpy as np

import pytest

from oracle import codec, fast, mca, opset as O

C = O.CONST
V0, V1 = O.VAR0, O.VAR0 + 1


def genotype(tokens, consts, height=4):
    ops = np.full(2 ** (height + 1) - 1, -1, dtype=np.int8)
    ops[: len(tokens)] = tokens
    cs = np.zeros(2 ** height, dtype=np.float32)
    cs[: len(consts)] = consts
    return codec.decode_one(ops, cs, height)


def run(progs, X, y, **kw):
    gs, cs = zip(*[genotype(t, c) for t, c in progs])
    return mca.flags(np.stack(gs), np.stack(cs), 4, X, y, **kw)


def test_flags():
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (2, 2000)).astype(np.float32)
    g = np.float32(O.GUARD)
    X[1, 7] = 2 * g                                   # x1 - GUARD == GUARD exactly
    y = (X[0] * X[1] + np.sin(X[0])).astype(np.float32)
    progs = [
        ([V0, V1, O.MUL, V0, O.SIN, O.ADD], []),             # the target: fine
        ([V0, V1, C, O.SUB, O.DIV], [O.GUARD]),              # guard input at its threshold
        ([V0, C, O.ADD, C, O.SUB], [1e4, 1e4]),              # cancellation at float32
        ([V0, O.SQ, V1, O.ADD], []),                         # fine
    ]
    f = run(progs, X, y)
    assert f.tolist() == [False, True, True, False]
    f64 = run(progs, X, y, precision="f64", rtol=1e-12)
    assert f64[0] == False and f64[3] == False and f64[1] == True


@pytest.mark.parametrize("impl", [mca, fast], ids=["numpy", "c"])
def test_gradient_branch_flags_a_cancelling_gradient(impl):
    """At the least-squares optimum of c in x0 + c sin(x1) the gradient is a
    sum of terms of both signs that cancel to about the rounding of c: a
    one-ulp perturbation of the node values moves it by far more than its
    tolerance, so with_grad flags it.  Far from the optimum (c = 2) the same
    tree is benign, and the fitness alone is well conditioned in both."""
    rng = np.random.default_rng(11)
    N = 3000
    X = rng.uniform(-2, 2, (2, N))
    y = X[0] + 0.5 * np.sin(X[1]) + 0.1 * rng.standard_normal(N)
    X32, y32 = X.astype(np.float32), y.astype(np.float32)
    Xd, yd = X32.astype(np.float64), y32.astype(np.float64)
    # optimum of c for the raw MSE (no linear scaling): least squares of
    # y - x0 on sin(x1), rounded to float32
    s = np.sin(Xd[1])
    c_opt = float(np.float32(np.dot(s, yd - Xd[0]) / np.dot(s, s)))
    progs = [([V0, C, V1, O.SIN, O.MUL, O.ADD], [c_opt]), ([V0, C, V1, O.SIN, O.MUL, O.ADD], [2.0])]
    kw = dict(linear_scaling=False, n=8)
    fg = run(progs, X32, y32, with_grad=True, **kw)
    ff = run(progs, X32, y32, with_grad=False, **kw)
    assert fg.tolist() == [True, False]
    assert ff.tolist() == [False, False]
    gs, cs = zip(*[genotype(t, c) for t, c in progs])
    sens = impl.sensitivity(np.stack(gs), np.stack(cs), 4, X32, y32, with_grad=True, **kw)
    from oracle import grad as GR
    g_opt = GR.gradient(gs[0], cs[0], 4, X32, y32, linear_scaling=False)[1]
    g_far = GR.gradient(gs[1], cs[1], 4, X32, y32, linear_scaling=False)[1]
    assert sens[0]["grad_spread"] > 1e-6 * abs(g_opt[0])        # cancelling: spread ~ |g|
    assert sens[1]["grad_spread"] < 1e-6 * abs(g_far[0])        # benign: spread ~ u |g|
    assert sens[0]["fit_spread"] < 1e-6 * sens[0]["fitness"]


@pytest.mark.parametrize("impl", [mca, fast], ids=["numpy", "c"])
def test_exp_clamp_and_pow_decisions(impl):
    """decision_inputs of exp is its argument against the clamp; of pow, the
    base against the guard and b ln|a| (0 where guarded) against the clamp.
    A program whose exp argument or pow exponent product sits on the clamp is
    near a decision; moving the thresholds changes the decision (the
    threshold-shifted runs flip it), and the spread reports the jump."""
    a = np.array([80.0, -79.0, 1e-7, 2.0])
    b = np.array([1.0, 1.0, 3.0, 80.0 / np.log(2.0)])
    (arr, thr), = O.decision_inputs(O.EXP, a, None)
    assert thr == O.CLAMP and np.array_equal(arr, a)
    (ga, gthr), (t, cthr) = O.decision_inputs(O.POW, a, b)
    assert gthr == O.GUARD and cthr == O.CLAMP and np.array_equal(ga, a)
    np.testing.assert_allclose(t, [80.0 * 0 + np.log(80.0), -0.0 + 1.0 * np.log(79.0), 0.0, 80.0])
    assert t[2] == 0.0                                          # guarded base: no exponent decision
    rng = np.random.default_rng(2)
    N = 500
    X = np.stack([rng.uniform(0.5, 1.0, N), np.full(N, 80.0), np.full(N, 2.0)]).astype(np.float32)
    y = X[0].astype(np.float32)
    progs = [([V0, O.VAR0 + 1, O.ADD, O.VAR0 + 1, O.EXP, O.ADD], []),   # exp(80): on the clamp
             ([V0, O.VAR0 + 2, C, O.POW, O.ADD], [80.0 / np.log(2.0)]),  # 2^(80/ln2) = e^80
             ([V0, O.VAR0 + 2, O.EXP, O.ADD], [])]                      # exp(2): far from it
    gs, cs = zip(*[genotype(t, c) for t, c in progs])
    sens = impl.sensitivity(np.stack(gs), np.stack(cs), 4, X, y, n=2)
    assert sens[0]["near"] and sens[1]["near"] and not sens[2]["near"]
    f = run(progs, X, y, n=2)
    assert f.tolist() == [True, True, False]


@pytest.mark.parametrize("impl", [mca, fast], ids=["numpy", "c"])
def test_threshold_shift_takes_the_other_decision(impl):
    """x0 / x1 with x1 = 1.00005 G on one row: the divisor is a terminal, so no
    perturbation of the node results reaches the guard, but the run with the
    guard raised by the window (1e-4) takes the guarded branch on that row:
    the individual counts as flipped and its fitness spread is the jump."""
    rng = np.random.default_rng(4)
    N = 400
    X = rng.uniform(1, 2, (2, N)).astype(np.float32)
    X[1, 3] = np.float32(1.00005 * O.GUARD)
    y = X[0].astype(np.float32)
    assert O.GUARD < float(X[1, 3]) < O.GUARD * (1 + 1e-4)
    g, gc = genotype([V0, V1, O.DIV], [])
    s = impl.sensitivity(g[None], gc[None], 4, X, y, n=2, window=1e-4)[0]
    assert s["near"] and s["flipped"] and s["fit_spread"] > 1e-3 * s["fitness"]
    # with the row moved away from the guard: nothing flips, the spread is rounding
    X[1, 3] = np.float32(1.5)
    s = impl.sensitivity(g[None], gc[None], 4, X, y, n=2, window=1e-4)[0]
    assert not s["near"] and not s["flipped"] and s["fit_spread"] < 1e-5 * s["fitness"]


def test_slope_spread_shows_a_variance_lost_against_the_mean():
    """b = S_py / S_pp: with p = x0 + 1e4 the binary32 rounding of p is about
    1e4 * 2^-24 of std(p), so the slope is known only to a few parts in 1e4;
    with p = x0 it is known to about the unit roundoff."""
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (2, 3000)).astype(np.float32)
    y = (2 * X[0] + 0.1 * X[1]).astype(np.float32)
    progs = [([V0], []), ([V0, C, O.ADD], [1e4])]
    gs, cs = zip(*[genotype(t, c) for t, c in progs])
    sens = mca.sensitivity(np.stack(gs), np.stack(cs), 4, X, y, n=6)
    b = [abs(s["b_spread"]) for s in sens]
    assert b[0] < 1e-6 * 2.0 and 1e-5 * 2.0 < b[1] < 1e-2 * 2.0
    assert sens[1]["a_spread"] > 1e4 * sens[1]["b_spread"] / 10   # a = ybar - b pbar
