"""The conditioning flags separate well- from ill-conditioned individuals."""
import numpy as np

from oracle import codec, mca, opset as O

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
