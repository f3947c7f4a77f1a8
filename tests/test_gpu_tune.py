"""The autotuner: it times launch shapes on the given inputs, keeps the fastest
for the problem class, writes and re-reads its file, and the tuned calls still
pass the parity gate against the oracle."""
import numpy as np
import pytest

import paper_2605_30954_amd as gg
from parity_util import (gate_fitness, gate_gradients, log, make_inputs, oracle_flags,
                         oracle_gradients, oracle_scores, to_device)
from synth import get_config

pytestmark = pytest.mark.gpu


def test_autotune_then_parity(tmp_path):
    cfg = get_config(2)
    M, N = 96, 30011
    log(f"[case] autotune cfg2 M={M} N={N}")
    d = make_inputs(cfg, M, N, salt=5)
    ops, cs, X, y = to_device(d)
    path = tmp_path / "tune.json"
    desc = gg.autotune(ops, cs, X, y, with_grad=True, cache_path=str(path), trials=1)
    log(f"[tune] {desc}")
    assert desc.startswith("forward K=") and "adjoint Kmask=" in desc
    assert gg.load_tuning(str(path)) >= 2
    fit, grad, st = gg.grad_consts(ops, cs, X, y, return_status=True)
    fit, grad, st = fit.cpu().numpy(), grad.cpu().numpy(), st.cpu().numpy()
    idx = list(range(M))
    vy = float(np.var(d["y"].astype(np.float64)))
    fl = oracle_flags(d, idx, "f32", with_grad=True)
    gate_fitness(fit, st, oracle_scores(d, idx), fl, vy, "f32", "tuned cfg2")
    rep = gate_gradients(grad, st, oracle_gradients(d, idx), fl, vy, what="tuned cfg2")
    assert rep["compared"] >= M // 2
