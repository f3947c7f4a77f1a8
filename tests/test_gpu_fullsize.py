"""Parity at the workloads' full sizes.

Each workload runs at its full M and N (cfg2 in the launch configuration the
benchmark times: autotuned shapes, graph replay on a non-default stream).  The
oracle cannot evaluate a whole batch at these sizes, so it checks a seeded
sample of programs one by one (fitness, status and the constant gradient,
gated as everywhere else; the Monte-Carlo conditioning check uses fewer
repetitions here), and every program of the batch is checked against
properties that hold at any size: status 0 exactly when the fitness is finite,
0 <= LS-MSE <= Var(y), NMSE = fitness / Var(y), a zero gradient past each
program's last constant, and bitwise-repeatable results."""
import numpy as np
import pytest

import paper_2605_30954_amd as gg
from parity_util import (gate_fitness, gate_gradients, log, make_inputs, oracle_flags,
                         oracle_gradients, oracle_scores, to_device)
from synth import get_config

pytestmark = pytest.mark.gpu


def _properties(fit, aux, st, grad, nc, vy):
    ok = st == 0
    assert np.array_equal(np.isfinite(fit), ok)
    assert np.all(fit[ok] >= 0.0) and np.all(fit[ok] <= vy * (1 + 1e-9))
    np.testing.assert_allclose(aux[ok, 3], fit[ok] / vy, rtol=1e-12)   # Var(y) summed in another order
    if grad is not None:
        C = grad.shape[1]
        past = np.arange(C)[None, :] >= nc[:, None]
        assert np.all(grad[past] == 0.0)
        assert np.all(grad[~ok] == 0.0)


def _run(cid, n_sample, mca_n, with_grad, tune, short_only=False, seed=0):
    import torch
    cfg = get_config(cid)
    log(f"[case] full size cfg{cid} M={cfg.M} N={cfg.N} grad={with_grad} tune={tune}")
    d = make_inputs(cfg, cfg.M, cfg.N, salt=0)
    ops, cs, X, y = to_device(d)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        if tune:
            log(f"[tune] {gg.autotune(ops, cs, X, y, with_grad=with_grad, trials=1)}")
        if with_grad:
            r1 = gg.grad_consts(ops, cs, X, y, return_aux=True, return_status=True)
            r2 = gg.grad_consts(ops, cs, X, y, return_aux=True, return_status=True)  # replay
            fit, grad, aux, st = [t.cpu().numpy() for t in r2]
            assert np.array_equal(r1[0].cpu().numpy(), fit, equal_nan=True)
            assert np.array_equal(r1[1].cpu().numpy(), grad, equal_nan=True)
        else:
            r1 = gg.eval_batch(ops, cs, X, y, return_aux=True, return_status=True)
            r2 = gg.eval_batch(ops, cs, X, y, return_aux=True, return_status=True)
            fit, aux, st = [t.cpu().numpy() for t in r2]
            grad = None
            assert np.array_equal(r1[0].cpu().numpy(), fit, equal_nan=True)
    s.synchronize()
    vy = float(np.var(d["y"].astype(np.float64)))
    _properties(fit, aux, st, grad, d["nc"].astype(np.int64), vy)
    rng = np.random.default_rng([cid, 77, seed])
    pool = np.arange(cfg.M)
    if short_only:   # oracle cost grows with the program length at N = 1e7
        pool = pool[d["ln"] <= 9]
    idx = sorted(rng.choice(pool, size=min(n_sample, pool.size), replace=False).tolist())
    fl = oracle_flags(d, idx, "f32", with_grad=with_grad, n=mca_n)
    ref = oracle_scores(d, idx)
    rep = gate_fitness(fit[idx], st[idx], ref, fl, vy, "f32", f"full cfg{cid}")
    if with_grad:
        gate_gradients(grad[idx], st[idx], oracle_gradients(d, idx), fl, vy, what=f"full cfg{cid}")
    return rep


@pytest.mark.timeout(600)
def test_cfg2_full_size_bench_configuration():
    rep = _run(2, n_sample=24, mca_n=4, with_grad=True, tune=True)
    assert rep["gated"] >= 12


@pytest.mark.timeout(600)
def test_cfg3_full_size_mixed_heights():
    rep = _run(3, n_sample=8, mca_n=3, with_grad=False, tune=False)
    assert rep["gated"] >= 4


@pytest.mark.timeout(600)
def test_cfg4_full_size_gradients():
    rep = _run(4, n_sample=8, mca_n=3, with_grad=True, tune=False)
    assert rep["gated"] >= 3


@pytest.mark.timeout(900)
def test_cfg5_full_size_large_templates():
    rep = _run(5, n_sample=6, mca_n=2, with_grad=False, tune=False, short_only=True)
    assert rep["gated"] >= 1
