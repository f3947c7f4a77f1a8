"""GPU parity of the constant gradient (reverse mode on the device) against the
oracle's forward-mode gradient, against central finite differences, and
through torch.autograd."""
import numpy as np
import pytest

import paper_2605_30954_amd as gg
from oracle import grad as OG
from parity_util import (gate_fitness, gate_gradients, log, make_inputs, oracle_flags,
                         oracle_gradients, oracle_scores, partial_peak, to_device)
from synth import get_config

pytestmark = pytest.mark.gpu


def run_grad(cid, M, N, linear_scaling=True, plain=False, salt=1, min_gated=None):
    min_gated = M // 3 if min_gated is None else min_gated
    cfg = get_config(cid)
    log(f"[case] grad cfg{cid} M={M} N={N} ls={linear_scaling} plain={plain}")
    d = make_inputs(cfg, M, N, salt)
    ops, cs, X, y = to_device(d)
    fit, grad, st = gg.grad_consts(ops, cs, X, y, linear_scaling=linear_scaling, plain=plain,
                                   return_status=True)
    fit, grad, st = fit.cpu().numpy(), grad.cpu().numpy(), st.cpu().numpy()
    idx = list(range(M))
    vy = float(np.var(d["y"].astype(np.float64)))
    fl = oracle_flags(d, idx, "f32", linear_scaling, with_grad=True)
    ref = oracle_scores(d, idx, linear_scaling)
    gate_fitness(fit, st, ref, fl, vy, "f32", f"grad-call fitness cfg{cid}")
    refs = oracle_gradients(d, idx, linear_scaling)
    rep = gate_gradients(grad, st, refs, fl, vy, what=f"cfg{cid} ls={linear_scaling} plain={plain}")
    assert rep["compared"] >= min_gated
    # per-row partials are float32: a gradient may be non-finite only where a
    # true per-row partial comes within a few decades of the float32 range
    nonfin = [m for m in range(M) if st[m] == 0 and not np.all(np.isfinite(grad[m]))]
    peaks = {m: partial_peak(d, m) for m in nonfin}
    log(f"[grad] non-finite gradients: {len(nonfin)} {peaks}")
    assert all(v >= 1e30 for v in peaks.values()), peaks
    return d, grad, st, refs, fl, vy


def test_cfg4_gradients_linear_scaling():
    run_grad(4, 64, 12000)


def test_cfg4_gradients_raw_mse():
    run_grad(4, 48, 9000, linear_scaling=False)


def test_cfg2_gradients():
    run_grad(2, 64, 10007)


@pytest.mark.parametrize("M", [1, 2, 3])
def test_gradients_tiny_batches(M):
    """Batches of fewer than four programs (the tier counts and the path
    tier's fallback flags share one workspace region)."""
    run_grad(4, M, 5000, salt=2, min_gated=0)


def test_cfg5_gradients_full_operator_set():
    # many random height-7 programs over all 11 operators have gradients that a
    # one-ulp perturbation of the node values moves by more than the plain
    # gate: their tolerance includes that measured spread
    run_grad(5, 64, 3001, min_gated=32)


def test_plain_adjoint_matches_fused():
    """The plain form (one launch per individual, the block's waves sharing
    it) and the fused form (class kernels over the batch) both within the
    oracle gate; the fused form is bitwise repeatable.  The two sum the rows
    in different groupings, so they are compared through the oracle rather
    than bitwise to each other."""
    cfg = get_config(4)
    M = 32
    d = make_inputs(cfg, M, 9000, salt=4)
    ops, cs, X, y = to_device(d)
    f1, g1, s1 = gg.grad_consts(ops, cs, X, y, return_status=True)
    f2, g2, s2 = gg.grad_consts(ops, cs, X, y, plain=True, return_status=True)
    f3, g3 = gg.grad_consts(ops, cs, X, y)
    assert np.array_equal(g1.cpu().numpy(), g3.cpu().numpy())   # bitwise repeatable
    idx = list(range(M))
    vy = float(np.var(d["y"].astype(np.float64)))
    fl = oracle_flags(d, idx, "f32", True, with_grad=True)
    refs = oracle_gradients(d, idx, True)
    for what, g, st in (("fused", g1, s1), ("plain", g2, s2)):
        g, st = g.cpu().numpy(), st.cpu().numpy()
        rep = gate_gradients(g, st, refs, fl, vy, what=f"cfg4 {what}")
        assert rep["compared"] >= 16
        nonfin = [m for m in range(M) if st[m] == 0 and not np.all(np.isfinite(g[m]))]
        assert all(partial_peak(d, m) >= 1e30 for m in nonfin), (what, nonfin)


def test_gradient_against_central_differences():
    """GPU gradient vs FP64 central differences (h = 1e-4) of the oracle's
    fitness, for every individual whose status is 0; constants next to a kink
    (FD at h and h/2 disagree) are skipped.  The tolerance adds the binary32
    rounding of the gradient's terms and its measured sensitivity, as the
    parity gate does."""
    cfg = get_config(4)
    d = make_inputs(cfg, 24, 6000, salt=9)
    ops, cs, X, y = to_device(d)
    fit, grad, st = gg.grad_consts(ops, cs, X, y, return_status=True)
    grad = grad.cpu().numpy()
    vy = float(np.var(d["y"].astype(np.float64)))
    sens = oracle_flags(d, list(range(24)), "f32", with_grad=True)
    refs = oracle_gradients(d, list(range(24)))
    checked = 0
    for m in range(24):
        gs = sens[m]["grad_spread"]
        if st[m].item() != 0 or gs is None or not np.isfinite(gs):
            continue
        f1 = OG.fd_gradient(d["genes"][m], d["gc"][m], 5, d["X"], d["y"], h=1e-4)
        f2 = OG.fd_gradient(d["genes"][m], d["gc"][m], 5, d["X"], d["y"], h=5e-5)
        if f1.size == 0:
            continue
        sc = float(np.max(np.abs(f1)))
        if np.max(np.abs(f1 - f2)) > 1e-6 * sc + 1e-12 * vy:
            continue
        tol = 2e-5 * sc + 1e-10 * vy + 4 * 2.0 ** -24 * float(np.max(refs[m][0]["gabs"])) + 3 * gs
        assert np.max(np.abs(grad[m, : f1.size] - f1)) <= tol, m
        checked += 1
    log(f"[fd] checked {checked} of 24")
    assert checked >= 12


def test_autograd_function():
    import torch
    cfg = get_config(4)
    d = make_inputs(cfg, 16, 5000, salt=2)
    ops, cs, X, y = to_device(d)
    c = cs.clone().requires_grad_(True)
    f = gg.GPGOMEAFitness.apply(c, ops, X, y)
    w = torch.linspace(0.5, 2.0, 16, dtype=torch.float64, device=f.device)
    (f * w).sum().backward()
    fit, grad = gg.grad_consts(ops, cs, X, y)
    ok = torch.isfinite(fit)
    want = (w[:, None] * grad).float()
    assert torch.allclose(c.grad[ok], want[ok], rtol=1e-6, atol=0)
    assert torch.equal(f, fit)


def test_clamped_exp_chain_gradient():
    """exp(exp(c / x0)) * x1 with c / x0 near the clamp of exp: where the inner
    exp is not clamped, its partial times d(c / x0)/dc (about 5e34 * 8e4)
    exceeds the binary32 range, while the outer exp is clamped on every row
    (its partial is 0).  The exact gradient is 0, and it must come out as 0,
    not NaN: a zero local partial ends the derivative path whatever the
    product below it holds.  The second program (c halved) reaches the same
    zero partial without any overflow."""
    import torch
    rng = np.random.default_rng(7)
    N = 4096
    X = np.stack([rng.uniform(1.2e-5, 1.3e-5, N), rng.standard_normal(N)]).astype(np.float32)
    y = (2.0 * X[1] + 0.1 * rng.standard_normal(N)).astype(np.float32)
    ops = np.full((2, 7), -1, np.int8)
    ops[:] = [32, 64, 3, 8, 8, 65, 2]   # c x0 / exp exp x1 *
    cs = np.array([[1e-3], [0.5e-3]], np.float32)
    log(f"[case] clamped exp chain M=2 N={N}")
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(a).to(dev)
    fit, grad, st = gg.grad_consts(t(ops), t(cs), t(X), t(y), return_status=True)
    fit, grad, st = fit.cpu().numpy(), grad.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0), st
    assert np.all(np.isfinite(fit)), fit
    assert np.array_equal(grad, np.zeros_like(grad)), grad


def test_gradient_graph_replays_match_eager():
    """A captured gradient call replayed several times, with eager calls, other
    work on the stream and synchronisations in between: every replay equals
    the eager result bitwise (the class kernels append fallen-back entries to
    the binary64 pass's lists with atomics; the partials must not depend on
    that order)."""
    import torch
    cfg = get_config(2)
    d = make_inputs(cfg, 256, 30011, salt=5)
    ops, cs, X, y = to_device(d)
    log("[case] grad graph replays cfg2 M=256 N=30011")
    s = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(s):
        eager = gg.grad_consts(ops, cs, X, y, graph=False, return_status=True)
        for k in range(4):
            outs.append(gg.grad_consts(ops, cs, X, y, return_status=True))  # capture, then replays
            junk = torch.randn(1 << 20, device="cuda:0") * float(k + 1)      # other work on the stream
            outs.append(gg.grad_consts(ops, cs, X, y, graph=False, return_status=True))
            s.synchronize()
            del junk
    s.synchronize()
    ref = [t.cpu().numpy() for t in eager]
    for o in outs:
        for a, b in zip(ref, [t.cpu().numpy() for t in o]):
            assert np.array_equal(a, b, equal_nan=True)
