"""Edge cases of the HIP path: ragged and tiny row counts, one individual,
single-token programs, non-finite data, malformed programs, the largest
templates (height 8, 511 tokens) and generating-formula trees."""
import numpy as np
import pytest

import paper_2605_30954_amd as gg
from oracle import codec as OC, fitness as OF, opset as O, tree as OT
from parity_util import log
from synth import get_config, make_dataset, sample_population

pytestmark = pytest.mark.gpu

V = [O.VAR0 + k for k in range(16)]
C = O.CONST


def dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in arrs]


def programs(progs, L=31, Cm=16):
    ops = np.full((len(progs), L), -1, np.int8)
    cs = np.zeros((len(progs), Cm), np.float32)
    for i, (t, c) in enumerate(progs):
        ops[i, : len(t)] = t
        c = list(c)[:Cm]  # a program may name more constants than the list holds
        cs[i, : len(c)] = c
    return ops, cs


def oracle_of(ops, cs, X, y, ls=True, rng="f32", height=6):
    out = []
    for i in range(len(ops)):
        g, gc = OC.decode_one(ops[i], cs[i], height)
        p = OT.evaluate(g, gc, height, X.astype(np.float64), rng=rng)
        out.append(OF.score(p, y, ls))
    return out


@pytest.mark.parametrize("N", [1, 2, 63, 64, 65, 511, 512, 513, 2049, 4097])
def test_ragged_row_counts(N):
    log(f"[case] ragged N={N}")
    rng = np.random.default_rng(N)
    X = rng.uniform(-2, 2, (3, N)).astype(np.float32)
    y = (X[0] * X[1] - np.cos(X[2])).astype(np.float32)
    progs = [([V[0], V[1], O.MUL], []), ([V[0], O.SIN, C, O.ADD], [0.5]),
             ([V[2], O.COS, V[0], V[1], O.MUL, O.SUB], []), ([C], [1.25])]
    ops, cs = programs(progs)
    for ls in (True, False):
        f, st = gg.eval_batch(*dev(ops, cs, X, y), linear_scaling=ls, return_status=True)
        ref = oracle_of(ops, cs, X, y, ls)
        for i, r in enumerate(ref):
            assert st[i].item() == r["status"]
            vy = float(np.var(y.astype(np.float64)))
            assert abs(f[i].item() - r["fitness"]) <= 1e-5 * abs(r["fitness"]) + 1e-10 * vy + 1e-30, (N, i)


@pytest.mark.parametrize("N", [1, 2, 63, 65, 257, 513, 2049])
def test_ragged_row_counts_gradients(N):
    """Constant gradients at tiny and ragged row counts (rows past the last
    one are masked in the forward and in every adjoint sink), against the
    oracle's forward-mode gradient; error bound relative to gabs, the sum of
    the per-row terms' magnitudes, plus 1e-12 absolute (targets are O(1): two
    rows are fitted exactly, so the residuals are rounding alone)."""
    from oracle import grad as OG
    log(f"[case] ragged gradient N={N}")
    rng = np.random.default_rng(100 + N)
    X = rng.uniform(-2, 2, (3, N)).astype(np.float32)
    y = (X[0] * X[1] - np.cos(X[2])).astype(np.float32)
    progs = [([V[0], C, O.ADD, O.SIN], [0.3]),                   # sin(x0 + c)
             ([C, V[1], O.MUL, V[2], O.COS, O.ADD], [1.7]),       # c x1 + cos x2
             ([V[0], C, O.MUL, O.EXP, V[1], C, O.SUB, O.MUL], [0.4, 0.9]),
             ([V[0], V[1], O.MUL, C, O.DIV, V[2], C, O.ADD, O.SQ, O.ADD], [1.3, -0.2])]
    ops, cs = programs(progs)
    f, g, st = gg.grad_consts(*dev(ops, cs, X, y), return_status=True)
    f, g, st = f.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    for i in range(len(progs)):
        genes, gc = OC.decode_one(ops[i], cs[i], 6)
        s, gr = OG.gradient(genes, gc, 6, X, y, linear_scaling=True, rng="f32")
        assert st[i] == s["status"], (N, i)
        nc = len(gr)
        assert np.all(g[i, nc:] == 0.0)
        for j in range(nc):
            tol = 1e-5 * s["gabs"][j] + 1e-6 * abs(gr[j]) + 1e-12
            assert abs(g[i, j] - gr[j]) <= tol, (N, i, j, g[i, j], gr[j], s["gabs"][j])


def test_single_individual_and_lone_terminals():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(2, 3000)).astype(np.float32)
    y = (2 * X[1] + 0.5).astype(np.float32)
    for progs in ([([V[1]], [])], [([C], [3.0])], [([V[0]], []), ([V[1]], []), ([C], [-1.0])]):
        ops, cs = programs(progs)
        f, aux, st = gg.eval_batch(*dev(ops, cs, X, y), return_aux=True, return_status=True)
        ref = oracle_of(ops, cs, X, y)
        for i, r in enumerate(ref):
            assert st[i].item() == 0
            assert f[i].item() == pytest.approx(r["fitness"], rel=1e-5, abs=1e-9)
    # x1 fits y = 2 x1 + 0.5 exactly after scaling: a = 0.5, b = 2
    ops, cs = programs([([V[1]], [])])
    f, aux = gg.eval_batch(*dev(ops, cs, X, y), return_aux=True)
    assert f.item() < 1e-10
    assert aux[0, 0].item() == pytest.approx(0.5, rel=1e-5) and aux[0, 1].item() == pytest.approx(2.0, rel=1e-5)


def test_nonfinite_data_and_overflow():
    rng = np.random.default_rng(6)
    X = rng.uniform(1, 2, (2, 5000)).astype(np.float32)
    y = X[0].astype(np.float32)
    X[1, 4321] = np.inf
    progs = [([V[0], V[1], O.ADD], []),             # touches the inf -> status 1
             ([V[0], O.SQ], []),                    # fine
             ([V[0], C, O.MUL, C, O.MUL], [1e30, 1e10]),   # overflows float32 -> status 1
             ([V[0], C, O.MUL, C, O.MUL, O.EXP], [1e30, 1e10])]  # exp(clamp(inf)) is finite
    ops, cs = programs(progs)
    f, st = gg.eval_batch(*dev(ops, cs, X, y), return_status=True)
    assert st.tolist() == [1, 0, 1, 0]
    assert np.isinf(f[0].item()) and np.isinf(f[2].item()) and np.isfinite(f[1].item())
    ref = oracle_of(ops, cs, X, y)
    assert [r["status"] for r in ref] == [1, 0, 1, 0]


def test_malformed_programs_get_status_2():
    rng = np.random.default_rng(7)
    X = rng.normal(size=(2, 1000)).astype(np.float32)
    y = X[0]
    progs = [([O.ADD], []), ([V[0], V[1]], []), ([V[5]], []), ([17], []), ([], []),
             ([C, C, O.ADD, C, O.ADD], [1, 2, 3]), ([V[0], V[1], O.DIV], [])]
    ops, cs = programs(progs, Cm=2)
    f, st = gg.eval_batch(*dev(ops, cs, X, y), return_status=True)
    assert st.tolist() == [2, 2, 2, 2, 2, 2, 0]
    assert all(np.isinf(f[i].item()) for i in range(6)) and np.isfinite(f[6].item())


def test_height8_templates_511_tokens():
    """Largest supported programs: full height-8 trees (511 tokens, 8 stack
    levels), the Exp. III template depth."""
    import dataclasses
    from synth.symbols import FUNCS_BASIC
    # binary operators only, so that "full" samples keep all 511 template slots
    cfg = dataclasses.replace(get_config(5), heights=(8,), funcs=FUNCS_BASIC)
    N = 3000
    X, y = make_dataset(cfg, N=N)
    genes, gc, hs = sample_population(cfg, M=16, salt=8)
    ops, cs, ln, nc = gg.encode(genes, gc, 8, 511, 256)
    assert ln.max() == 511
    f, st = gg.eval_batch(*dev(ops, cs, X, y), return_status=True)
    ref = OF.evaluate_population(genes, gc, 8, X, y)
    vy = float(np.var(y.astype(np.float64)))
    from oracle import mca
    from parity_util import gate_fitness
    sens = mca.sensitivity(genes, gc, 8, X, y, n=4)
    gate_fitness(f.cpu().numpy(), st.cpu().numpy(), ref, sens, vy, "f32", "height 8")


def test_generating_formula_tree_fits():
    """A tree equal to the generating formula reaches LS-MSE ~ 0 (noise-free
    cfg4 target; cfg1's target needs height 4 so a height-5 template is used)."""
    cfg = get_config(4)
    X, y = make_dataset(cfg, N=50000)
    t = [C, V[0], V[0], O.MUL, O.MUL, C, V[1], O.MUL, V[4], O.MUL, O.SUB, C, V[2], O.MUL, O.COS,
         O.ADD]
    ops, cs = programs([(t, [2.3, 0.7, 1.9])], L=63, Cm=32)
    for fp64 in (False, True):
        f, aux = gg.eval_batch(*dev(ops, cs, X, y), fp64_nodes=fp64, return_aux=True)
        assert aux[0, 3].item() <= (1e-10 if not fp64 else 1e-13), (fp64, aux[0, 3].item())
