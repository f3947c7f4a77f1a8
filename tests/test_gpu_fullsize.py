"""Parity at the workloads' full sizes.

Each workload runs at its full M and N in the launch configuration the
benchmark times: graph replay on a non-default stream, with the shipped MI355X
tuning file loaded (cfg2 also runs the autotuner).  The oracle checks a seeded
sample of programs one by one with its C implementation (oracle/fast.py, pinned
to the NumPy oracle): fitness, status and the constant gradient, each graded
with the gate plus three times the program's own measured sensitivity.  For
the height-7 workload the sample is the longest programs (every one of 128
tokens or more, and more of 64 or more) plus random ones.  Every program of the
batch is also checked against properties that hold at any size: status 0
exactly when the fitness is finite, 0 <= LS-MSE <= Var(y), NMSE =
fitness / Var(y), a zero gradient past each program's last constant, and
bitwise-repeatable results (a graph replay equals the first launch)."""
import os

import numpy as np
import pytest

import paper_2605_30954_amd as gg
from oracle import fast
from parity_util import check_properties, gate_fitness, gate_gradients, log, make_inputs, to_device
from synth import get_config

pytestmark = pytest.mark.gpu


def _sample(d, cid, n_rand, seed=0):
    rng = np.random.default_rng([cid, 77, seed])
    ln = d["ln"].astype(np.int64)
    idx = []
    if cid == 5:  # the long programs the workload is about
        idx += np.nonzero(ln >= 128)[0].tolist()
        long64 = np.nonzero((ln >= 64) & (ln < 128))[0]
        idx += sorted(long64[np.argsort(-ln[long64], kind="stable")][:4].tolist())
    rest = np.setdiff1d(np.arange(len(ln)), idx)
    idx += rng.choice(rest, size=min(n_rand, rest.size), replace=False).tolist()
    return sorted(set(int(i) for i in idx))


def _run(cid, n_rand, mca_n, with_grad, tune=False):
    import torch
    cfg = get_config(cid)
    log(f"[case] full size cfg{cid} M={cfg.M} N={cfg.N} grad={with_grad} tune={tune}")
    if os.path.exists(gg.TUNING_FILE):
        log(f"[tune] shipped file: {gg.load_tuning(gg.TUNING_FILE)} entries")
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
    del ops, cs, X, y, r1, r2
    vy = float(np.var(d["y"].astype(np.float64)))
    check_properties(fit, aux, st, grad, d["nc"].astype(np.int64), vy)
    idx = _sample(d, cid, n_rand)
    log(f"[sample] cfg{cid}: {len(idx)} programs, lengths {sorted(d['ln'][idx].tolist())}")
    sens = fast.sensitivity(d["genes"], d["gc"], d["hs"], d["X"], d["y"], n=mca_n, with_grad=with_grad,
                            indices=idx)
    refs = [fast.run(d["genes"][m], d["gc"][m], int(d["hs"][m]), d["X"], d["y"], with_grad=with_grad)
            for m in idx]
    ref = {k: np.array([r[k] for r in refs]) for k in ("fitness", "status")}
    rep = gate_fitness(fit[idx], st[idx], ref, sens, vy, "f32", f"full cfg{cid}")
    if with_grad:
        grep = gate_gradients(grad[idx], st[idx], [(r, r["grad"]) for r in refs], sens, vy,
                              what=f"full cfg{cid}")
        return rep, grep
    return rep, None


@pytest.mark.timeout(600)
def test_cfg2_full_size_autotuned():
    rep, grep = _run(2, n_rand=24, mca_n=4, with_grad=True, tune=True)
    assert rep["gated"] == 24 and grep["compared"] >= 12


@pytest.mark.timeout(600)
def test_cfg3_full_size_mixed_heights():
    rep, _ = _run(3, n_rand=10, mca_n=3, with_grad=False)
    assert rep["gated"] == 10


@pytest.mark.timeout(600)
def test_cfg4_full_size_gradients():
    rep, grep = _run(4, n_rand=10, mca_n=3, with_grad=True)
    assert rep["gated"] == 10 and grep["compared"] >= 5


@pytest.mark.timeout(900)
def test_cfg5_full_size_fused_fitness_and_gradient():
    """The benchmark's workload: 8192 height-7 programs over all 11 operators,
    1e7 rows of heavy-tailed targets, fused fitness + gradient."""
    rep, grep = _run(5, n_rand=2, mca_n=2, with_grad=True)
    assert rep["gated"] >= 8
    assert grep["compared"] + grep["status_sensitive"] >= 6
