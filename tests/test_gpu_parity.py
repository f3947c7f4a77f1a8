"""GPU parity: the HIP path (through the C ABI) against the float64 oracle on
every workload, at sizes the oracle finishes quickly, spanning several row
tiles, a ragged tail, both node precisions, both fitness kinds and both launch
forms (fused batch and one launch per individual)."""
import numpy as np
import pytest

from parity_util import (K_SPREAD, gate_fitness, log, make_inputs, oracle_flags, oracle_scores,
                         to_device)
from synth import get_config

pytestmark = pytest.mark.gpu

import paper_2605_30954_amd as gg  # noqa: E402


def run_case(cid, M, N, precision="f32", linear_scaling=True, plain=False, graph=True, salt=0):
    cfg = get_config(cid)
    log(f"[case] cfg{cid} M={M} N={N} {precision} ls={linear_scaling} plain={plain} graph={graph}")
    d = make_inputs(cfg, M, N, salt)
    ops, cs, X, y = to_device(d)
    fit, aux, st = gg.eval_batch(ops, cs, X, y, linear_scaling=linear_scaling,
                                 fp64_nodes=(precision == "f64"), plain=plain, graph=graph,
                                 return_aux=True, return_status=True)
    fit, aux, st = fit.cpu().numpy(), aux.cpu().numpy(), st.cpu().numpy()
    idx = list(range(M))
    ref = oracle_scores(d, idx, linear_scaling, precision)
    fl = oracle_flags(d, idx, precision, linear_scaling)
    vy = float(np.var(d["y"].astype(np.float64)))
    rep = gate_fitness(fit, st, ref, fl, vy, precision, f"cfg{cid} {precision} ls={linear_scaling}")
    return d, fit, aux, st, ref, fl, rep


def test_cfg1_fp32_linear_scaling():
    run_case(1, 64, 1000)


def test_cfg1_fp32_raw_mse():
    run_case(1, 64, 1000, linear_scaling=False)


def test_cfg1_fp64_nodes():
    run_case(1, 64, 1000, precision="f64")


def test_cfg1_plain_form():
    run_case(1, 64, 1000, plain=True)


def test_cfg2_fp32_several_tiles_ragged_tail():
    run_case(2, 256, 20011)


def test_cfg2_fp64_nodes():
    run_case(2, 128, 9001, precision="f64")


def test_cfg2_plain_form_raw():
    run_case(2, 64, 20011, plain=True, linear_scaling=False)


def test_cfg3_mixed_heights():
    run_case(3, 192, 12345)


def test_cfg4_fp32():
    run_case(4, 128, 15000)


def test_cfg5_fp32_full_operator_set():
    run_case(5, 48, 4099)


def test_cfg5_fp64_nodes():
    run_case(5, 24, 2000, precision="f64")


def test_aux_outputs_match_oracle():
    """Every status-0 individual's aux outputs, each graded like the fitness:
    rtol 1e-5 relative plus three times the individual's measured sensitivity
    of that output (the slope b = S_py / S_pp loses the digits that the
    prediction's variance loses against its mean, and the spread shows it)."""
    d, fit, aux, st, ref, sens, _ = run_case(2, 96, 7000)
    vy = float(np.var(d["y"].astype(np.float64)))
    sens_raw = oracle_flags(d, list(range(96)), "f32", linear_scaling=False)
    ok = (st == 0) & (ref["status"] == 0)
    assert ok.sum() > 50
    checked = 0
    for m in np.nonzero(ok)[0]:
        s, sr = sens[m], sens_raw[m]
        if not np.isfinite(s["fit_spread"]):
            continue
        checks = [("nmse", aux[m, 3], ref["nmse"][m], (1e-10 * vy + K_SPREAD * s["fit_spread"]) / vy),
                  ("mse", aux[m, 2], ref["mse"][m], 1e-10 * vy + K_SPREAD * sr["fit_spread"]),
                  ("b", aux[m, 1], ref["b"][m], K_SPREAD * s["b_spread"]),
                  ("a", aux[m, 0], ref["a"][m], 1e-10 * np.sqrt(vy) + K_SPREAD * s["a_spread"])]
        for what, got, want, extra in checks:
            assert abs(got - want) <= 1e-5 * abs(want) + extra, (m, what, got, want, extra)
        checked += 1
    log(f"[aux] {checked} individuals: NMSE, raw MSE, intercept and slope within the gate")
    assert checked > 50


def test_plain_and_fused_agree_and_are_deterministic():
    cfg = get_config(2)
    d = make_inputs(cfg, 128, 30000, salt=3)
    import torch
    ops, cs, X, y = to_device(d)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):   # captured graphs need a non-default stream
        r = [gg.eval_batch(ops, cs, X, y) for _ in range(3)]   # capture, then replays
        r.append(gg.eval_batch(ops, cs, X, y, graph=False))
        r.append(gg.eval_batch(ops, cs, X, y, plain=True))
    s.synchronize()
    f1, f2, f5, f3, f4 = [t.cpu().numpy() for t in r]
    assert np.array_equal(f1, f5, equal_nan=True)
    assert np.array_equal(f1, f2, equal_nan=True)          # bitwise repeatable
    assert np.array_equal(f1, f3, equal_nan=True)          # graph == direct launch
    fin = np.isfinite(f1)
    np.testing.assert_allclose(f4[fin], f1[fin], rtol=1e-9, atol=1e-12)
    assert np.array_equal(np.isfinite(f4), fin)


def test_forward_group_sizes_agree(tmp_path):
    """Groups of 16, 64 and 128 programs (the forward's largest) with a ragged
    last group: the oracle's gate for the largest, and bitwise the same
    fitness for all three (a program's sums do not depend on its group)."""
    cfg = get_config(2)
    M, N = 300, 5000
    d = make_inputs(cfg, M, N, salt=21)
    ops, cs, X, y = to_device(d)
    lcls = int(np.floor(np.log2(cfg.L_max + 1)))
    outs = {}
    for G in (16, 64, 128):
        path = str(tmp_path / f"fwd_{G}.json")
        with open(path, "w") as fh:
            fh.write('{"entries": [\n  {"table": "fwd", "fp64": 0, "Lcls": %d, "F": %d, "Ncls": %d, '
                     '"Mcls": %d, "grad": 0, "K": 8, "R": 512, "G": %d}\n]}\n'
                     % (lcls, cfg.F, int(np.log2(N)), int(np.log2(M)), G))
        assert gg.load_tuning(path) == 1
        log(f"[case] forward group size {G}, cfg2 M={M} N={N}")
        fit, st = gg.eval_batch(ops, cs, X, y, return_status=True)
        outs[G] = (fit.cpu().numpy(), st.cpu().numpy())
    for G in (16, 64):
        assert np.array_equal(outs[G][1], outs[128][1])
        assert np.array_equal(outs[G][0].view(np.uint64), outs[128][0].view(np.uint64)), G
    idx = list(range(M))
    vy = float(np.var(d["y"].astype(np.float64)))
    gate_fitness(outs[128][0], outs[128][1], oracle_scores(d, idx), oracle_flags(d, idx), vy, "f32",
                 "cfg2 forward groups of 128")
