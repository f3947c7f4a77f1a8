"""GPU parity of the gradient's work classes, the constant-free and guard edge
cases, and the graph cache, against the float64 oracle.

The gradient runs in path forward mode in one kernel per class of programs
(at most 4, 8, 16 or any number of constants, the last cut into chunks of 32;
an eight-slot class for programs needing more than four stack slots), with a
binary64 recomputation of the row spans whose binary32 chain-rule products
left the binary32 range.  Every program here is built so that it lands in a
known class; the oracle evaluates the decoded tree."""
import numpy as np
import pytest

import paper_2605_30954_amd as gg
from oracle import codec as OC, fitness as OF, grad as OG, opset as O, tree as OT
from parity_util import (gate_fitness, gate_gradients, log, make_inputs, oracle_flags,
                         oracle_gradients, oracle_scores, to_device)
from synth import get_config

pytestmark = pytest.mark.gpu

C = O.CONST
V = [O.VAR0 + k for k in range(16)]


def dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0") for a in arrs]


def product(k, F):
    return [C, V[k % F], O.MUL]


def balanced(parts, op=O.ADD):
    """Postfix of a balanced binary tree of `op` over the subtrees `parts`."""
    if len(parts) == 1:
        return parts[0]
    h = (len(parts) + 1) // 2
    return balanced(parts[:h], op) + balanced(parts[h:], op) + [op]


def left_chain(parts, op=O.ADD):
    out = parts[0]
    for q in parts[1:]:
        out = out + q + [op]
    return out


def pack(progs, L, Cm, rng):
    ops = np.full((len(progs), L), -1, np.int8)
    cs = np.zeros((len(progs), Cm), np.float32)
    for i, t in enumerate(progs):
        assert len(t) <= L
        ops[i, : len(t)] = t
        nc = sum(1 for s in t if s == C)
        cs[i, :nc] = rng.uniform(-1.0, 1.0, nc).astype(np.float32)
    return ops, cs


def oracle_grad_of(ops, cs, X, y, height, ls=True):
    out = []
    for i in range(len(ops)):
        g, gc = OC.decode_one(ops[i], cs[i], height)
        out.append(OG.gradient(g, gc, height, X, y, linear_scaling=ls, rng="f32"))
    return out


def check_against_oracle(ops, cs, X, y, height, what, ls=True, plain=False, rtol=1e-5):
    vy = float(np.var(y.astype(np.float64)))
    f, g, st = gg.grad_consts(*dev(ops, cs, X, y), linear_scaling=ls, plain=plain, return_status=True)
    f, g, st = f.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
    refs = oracle_grad_of(ops, cs, X, y, height, ls)
    for i, (s, gr) in enumerate(refs):
        assert st[i] == s["status"], (what, i)
        if s["status"]:
            continue
        assert abs(f[i] - s["fitness"]) <= rtol * abs(s["fitness"]) + 1e-10 * vy, (what, i, f[i], s["fitness"])
        nc = gr.size
        assert np.all(g[i, nc:] == 0.0), (what, i)
        if nc:
            tol = rtol * np.max(np.abs(gr)) + 1e-10 * vy + 4 * 2.0 ** -24 * np.max(s["gabs"])
            err = np.max(np.abs(g[i, :nc] - gr))
            assert err <= tol, (what, i, nc, err, tol)
    log(f"[classes] {what}: {len(ops)} programs within the gate")
    return f, g, st


def test_chunked_and_deep_programs():
    """40 constants in a shallow program (class of chunks of 32: two entries)
    and 64 constants in a program needing six stack slots (deep class, two
    entries), next to programs of every smaller class, 511-token stride."""
    rng = np.random.default_rng(31)
    F, N = 5, 3001
    X = rng.uniform(-1, 1, (F, N)).astype(np.float32)
    y = (np.sin(X[0]) + X[1] * X[2] - 0.5 * X[3]).astype(np.float32)
    groups = [balanced([product(10 * g + k, F) for k in range(10)]) for g in range(4)]
    shallow40 = left_chain(groups)                                   # need 4, 40 constants
    deep64 = balanced([product(k, F) for k in range(64)])             # need 6, 64 constants
    small = [balanced([product(k, F) for k in range(n)]) + [O.SIN] for n in (1, 3, 6, 12, 20)]
    progs = [shallow40, deep64] + small
    ops, cs = pack(progs, 511, 64, rng)
    log(f"[case] chunked/deep: lengths {[len(t) for t in progs]}")
    check_against_oracle(ops, cs, X, y, 8, "chunked+deep")
    check_against_oracle(ops, cs, X, y, 8, "chunked+deep plain", plain=True)


def test_flush_events_beyond_constant_count():
    """((c+x0)*(x1+x2))*((x0+x1)*(x2+x0)) has one constant but two flush
    events (the push of the constant-holding subtree and a merge-free
    product above it): the event list must hold every event, so the chain
    factor (x1+x2) is not lost.  With one constant column (C_max = 1)."""
    rng = np.random.default_rng(5)
    F, N = 3, 2048
    X = rng.uniform(-1, 1, (F, N)).astype(np.float32)
    y = (X[0] * X[1] + X[2]).astype(np.float32)
    t = [C, V[0], O.ADD, V[1], V[2], O.ADD, O.MUL, V[0], V[1], O.ADD, V[2], V[0], O.ADD, O.MUL, O.MUL]
    t2 = [V[0], V[1], O.ADD, V[2], V[0], O.ADD, O.MUL, C, V[0], O.ADD, V[1], V[2], O.ADD, O.MUL, O.MUL]
    ops, cs = pack([t, t2], 15, 1, rng)
    check_against_oracle(ops, cs, X, y, 4, "flush events, C_max=1")


def test_no_constants_batch():
    """C_max = 0: fitness as eval_batch, an empty gradient, fused and plain."""
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, (2, 4000)).astype(np.float32)
    y = (X[0] * X[1]).astype(np.float32)
    ops = np.full((3, 7), -1, np.int8)
    ops[0, :3] = [V[0], V[1], O.MUL]
    ops[1, :2] = [V[0], O.SIN]
    ops[2, :5] = [V[0], V[1], O.ADD, V[0], O.MUL]
    cs = np.zeros((3, 0), np.float32)
    for plain in (False, True):
        f0 = gg.eval_batch(*dev(ops, cs, X, y), plain=plain).cpu().numpy()
        f, g = gg.grad_consts(*dev(ops, cs, X, y), plain=plain)
        assert g.shape == (3, 0)
        assert np.array_equal(f.cpu().numpy(), f0)
    ref = [OF.score(OT.evaluate(*OC.decode_one(ops[i], cs[i], 3), 3, X.astype(np.float64)), y)
           for i in range(3)]
    for i in range(3):
        assert abs(f0[i] - ref[i]["fitness"]) <= 1e-5 * ref[i]["fitness"] + 1e-12


@pytest.mark.parametrize("kmask,R,G", [(0, 256, 4), (7, 512, 16), (4, 1024, 32), (3, 256, 64)])
def test_every_class_variant(kmask, R, G, tmp_path):
    """Each rows-per-lane choice of classes 0-2, tile and group size, on the
    height-5 and height-7 workloads (D = 4 programs, rolling program windows)."""
    for cid, M, N in ((4, 48, 3001), (5, 40, 2600)):
        cfg = get_config(cid)
        d = make_inputs(cfg, M, N, salt=13)
        ops, cs, X, y = to_device(d)
        lcls = int(np.floor(np.log2(cfg.L_max + 1)))
        path = str(tmp_path / f"tune_{cid}.json")
        with open(path, "w") as fh:
            fh.write('{"entries": [\n  {"table": "adj", "fp64": 0, "Lcls": %d, "F": %d, "Ncls": %d, '
                     '"Mcls": %d, "grad": 1, "K": %d, "R": %d, "G": %d}\n]}\n'
                     % (lcls, cfg.F, int(np.log2(N)), int(np.log2(M)), kmask, R, G))
        assert gg.load_tuning(path) == 1
        log(f"[case] class variant cfg{cid} Kmask={kmask} R={R} G={G}")
        f, g, st = gg.grad_consts(ops, cs, X, y, return_status=True)
        g, st = g.cpu().numpy(), st.cpu().numpy()
        idx = list(range(M))
        vy = float(np.var(d["y"].astype(np.float64)))
        fl = oracle_flags(d, idx, "f32", True, with_grad=True)
        rep = gate_gradients(g, st, oracle_gradients(d, idx, True), fl, vy,
                             what=f"cfg{cid} Kmask={kmask} R={R} G={G}")
        assert rep["compared"] >= M // 3


def test_guard_thresholds():
    """Inputs exactly at, one ulp below and one ulp above the protection
    threshold G (the binary32 number nearest 1e-6) of division, log and pow,
    and at the clamp of exp: the device takes the oracle's decision (a strict
    |v| < G guards; the clamp keeps +-80).  Raw MSE against y = 0 is p^2, so a
    wrong decision changes the fitness by orders of magnitude."""
    G = np.float32(O.GUARD)
    vals = [G, np.nextafter(G, np.float32(0)), np.nextafter(G, np.float32(1)), -G,
            -np.nextafter(G, np.float32(0)), np.float32(0)]
    progs = [[V[0], V[1], O.DIV],                    # 1000 / v or 1
             [V[1], O.LOG],                          # ln|v| or 0
             [V[1], C, O.POW]]                       # |v|^-1 or 0
    rng = np.random.default_rng(0)
    ops, cs = pack(progs, 3, 1, rng)
    cs[:] = -1.0
    for v in vals:
        X = np.array([[1000.0], [v]], np.float32)
        y = np.zeros(1, np.float32)
        f, st = gg.eval_batch(*dev(ops, cs, X, y), linear_scaling=False, return_status=True)
        f = f.cpu().numpy()
        for i in range(len(progs)):
            g_, gc_ = OC.decode_one(ops[i], cs[i], 2)
            p = OT.evaluate(g_, gc_, 2, X.astype(np.float64))
            ref = OF.score(p, y, linear_scaling=False)["fitness"]
            # binary32 log/exp carry about 1e-6 relative in |v|^-1 (squared here);
            # a wrong guard decision is off by six orders of magnitude
            assert abs(f[i] - ref) <= 1e-4 * abs(ref) + 1e-30, (float(v), i, f[i], ref)
    # exp's clamp: the gradient of mean(exp(c x)^2) in c is 2 exp(2cx) x inside
    # the clamp and 0 beyond it (c x = 80 exactly is inside)
    x = np.float32(1.0)
    for c, inside in ((80.0, True), (float(np.nextafter(np.float32(80), np.float32(100))), False)):
        X = np.array([[x]], np.float32)
        y = np.zeros(1, np.float32)
        ops1 = np.array([[C, V[0], O.MUL, O.EXP]], np.int8)
        cs1 = np.array([[c]], np.float32)
        f, g = gg.grad_consts(*dev(ops1, cs1, X, y), linear_scaling=False)
        g = g.cpu().numpy()[0, 0]
        if inside:
            want = 2.0 * np.exp(2 * 80.0)
            assert abs(g - want) <= 1e-5 * want, (g, want)
        else:
            assert g == 0.0, g


def test_graph_cache_changing_batch_size():
    """Graph replays over five batch sizes on the same buffers and with
    retained outputs: every result matches the oracle, graph results equal
    direct launches bitwise, and the cache holds one executable graph for the
    shape class (updated in place), never more than its bound."""
    import torch
    cfg = get_config(4)
    M, N = 96, 4099
    d = make_inputs(cfg, M, N, salt=21)
    ops, cs, X, y = to_device(d)
    vy = float(np.var(d["y"].astype(np.float64)))
    s = torch.cuda.Stream()
    gg.clear_graphs()
    kept = []
    with torch.cuda.stream(s):
        for m in (96, 17, 64, 3, 96, 40):
            r = gg.grad_consts(ops[:m], cs[:m], X, y, return_status=True)        # graph
            e = gg.grad_consts(ops[:m], cs[:m], X, y, graph=False, return_status=True)
            kept.append((m, r, e))
            assert gg.graph_count() == 1, gg.graph_count()
    s.synchronize()
    for m, r, e in kept:
        for a, b in zip(r, e):
            assert torch.equal(a.cpu(), b.cpu()) or np.array_equal(a.cpu().numpy(), b.cpu().numpy(), equal_nan=True)
    m, r, _ = kept[1]
    idx = list(range(m))
    fl = oracle_flags(d, idx, "f32", True, with_grad=True)
    gate_fitness(r[0].cpu().numpy(), r[2].cpu().numpy(), oracle_scores(d, idx), fl, vy, "f32", "graph M=17")
    gate_gradients(r[1].cpu().numpy(), r[2].cpu().numpy(), oracle_gradients(d, idx), fl, vy, what="graph M=17")
    # many calls with new outputs and other shapes: the cache stays bounded
    with torch.cuda.stream(s):
        for k in range(40):
            n = 1000 + 97 * k
            gg.eval_batch(ops[:8], cs[:8], X[:, :n].contiguous(), y[:n].contiguous())
    s.synchronize()
    assert 1 <= gg.graph_count() <= 16, gg.graph_count()


def test_binary64_redo_of_single_row_tiles():
    """x0 / (c - x1) with c just above x1 at three rows, where x0 = 1e28: the
    value stays in the binary32 range but d/dc = -x0 / (c - x1)^2 does not,
    so the binary32 sums of the row tiles holding those rows are left out and
    redone in binary64 (two of the rows share a span, in different tiles; the
    third is in another span).  400,000 rows give several tiles per span.  The
    overflowing rows dominate the gradient of the raw MSE (their residuals are
    6% of their values), so a tile lost or counted twice shows; with linear
    scaling the fit would absorb those rows and leave a cancelling sum.  One,
    10 and 20 constants (three work classes), fused and plain."""
    rng = np.random.default_rng(17)
    F, N = 3, 400_000
    X = rng.uniform(-1, 1, (F, N)).astype(np.float32)
    rows = [123_457, 124_057, 300_001]
    X[0, rows] = [1e28, 2e28, 3e28]
    X[1, rows] = np.float32(1.999998)
    x = X.astype(np.float64)
    y = (x[0] / (2.0 - x[1]) + 0.1 * x[2]).astype(np.float32)
    assert np.all(np.isfinite(y))
    trigger = [V[0], C, V[1], O.SUB, O.DIV]
    progs = [balanced([trigger] + [[C, V[2], O.MUL]] * n) for n in (0, 9, 19)]
    progs.append([C, V[2], O.MUL, C, O.ADD])                      # no overflow anywhere
    ops, cs = pack(progs, 511, 32, rng)
    cs[:3, 0] = np.float32(1.9999999)
    log(f"[case] tile-granular binary64 redo: N={N}, rows {rows}")
    f, g, st = check_against_oracle(ops, cs, X, y, 8, "single-row tile redo", ls=False)
    assert np.all(st == 0)
    assert np.all(np.isfinite(g)) and np.all(np.abs(g[:3, 0]) > 1e60)
    check_against_oracle(ops, cs, X, y, 8, "single-row tile redo, plain", ls=False, plain=True)
