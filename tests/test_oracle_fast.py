"""Pins of the oracle's C implementation (oracle/fast.py, ctree.c) against its
NumPy implementation, which tests/test_oracle_*.py pin to the paper, closed
forms and brute force: predictions, fitness, statuses, gradients, gradient
term magnitudes and the near-a-decision flags on every workload, both
fitness kinds, and the conditioning pins of the Monte-Carlo check."""
import numpy as np
import pytest

from oracle import fast, fitness as FT, grad as GR, mca, tree as TR
from synth import get_config, make_dataset, sample_population


@pytest.mark.parametrize("cid,M,N", [(1, 40, 500), (2, 40, 700), (3, 40, 600), (4, 40, 600), (5, 40, 500)])
@pytest.mark.parametrize("ls", [True, False])
def test_matches_numpy_oracle(cid, M, N, ls):
    cfg = get_config(cid)
    X, y = make_dataset(cfg, N=N, salt=7)
    genes, gc, hs = sample_population(cfg, M=M, salt=7)
    # tolerance: the binary64 sensitivity (libm and summation differ by ulps);
    # decisions: the binary32-range evaluation both sides run
    sens = mca.sensitivity(genes, gc, hs, X, y, precision="f64", n=2, linear_scaling=ls, with_grad=True)
    near32 = [s["near"] for s in mca.sensitivity(genes, gc, hs, X, y, precision="f32", n=0,
                                                  linear_scaling=ls)]
    X64 = X.astype(np.float64)
    for m in range(M):
        h = int(hs[m])
        s_np, g_np = GR.gradient(genes[m], gc[m], h, X, y, linear_scaling=ls, rng="f32")
        s_c = fast.run(genes[m], gc[m], h, X, y, linear_scaling=ls, rng="f32", return_p=True)
        p_np = TR.evaluate(genes[m], gc[m], h, X64, rng="f32")
        fin = np.isfinite(p_np)
        assert np.array_equal(fin, np.isfinite(s_c["p"])), (cid, m)
        # row by row where binary64 evaluation is well conditioned (a huge
        # argument of sin/cos is not: one ulp of it moves the result anywhere)
        well = sens[m]["fit_spread"] <= 1e-10 * abs(s_np["fitness"]) and not sens[m]["near"]
        scale = float(np.max(np.abs(p_np[fin]), initial=0.0))
        assert not well or np.allclose(s_c["p"][fin], p_np[fin], rtol=1e-9, atol=1e-9 * scale), (cid, m)
        assert s_c["status"] == s_np["status"], (cid, m)
        near_c = s_c["near"] or (s_c["status"] == 0 and
                                 0 < s_c["vp"] <= 1e2 * FT.DEGENERATE_RTOL * max(s_c["pbar"] ** 2, 1e-300))
        assert near_c == near32[m], (cid, m)
        if s_np["status"] != 0:
            assert np.isinf(s_c["fitness"])
            continue
        f = s_np["fitness"]
        tol = 1e-9 * abs(f) + 1e-14 * float(np.var(y.astype(np.float64))) + 3 * sens[m]["fit_spread"]
        assert abs(s_c["fitness"] - f) <= tol, (cid, m, s_c["fitness"], f)
        assert g_np.size == s_c["grad"].size
        if g_np.size:
            gs = sens[m]["grad_spread"]
            tol = 1e-9 * np.max(np.abs(g_np)) + 1e-12 * np.max(s_np["gabs"]) + 3 * gs
            assert np.max(np.abs(s_c["grad"] - g_np)) <= tol, (cid, m)
            np.testing.assert_allclose(s_c["gabs"], s_np["gabs"], rtol=1e-9, atol=1e-300 + 3 * gs)


def test_threads_do_not_change_results_beyond_rounding():
    cfg = get_config(5)
    X, y = make_dataset(cfg, N=20000, salt=3)
    genes, gc, hs = sample_population(cfg, M=6, salt=3)
    for m in range(6):
        a = fast.run(genes[m], gc[m], 7, X, y, nthreads=1)
        b = fast.run(genes[m], gc[m], 7, X, y, nthreads=7)
        assert a["status"] == b["status"]
        if a["status"] == 0:
            assert abs(a["fitness"] - b["fitness"]) <= 1e-13 * abs(a["fitness"])
            np.testing.assert_allclose(a["grad"], b["grad"], rtol=1e-11, atol=1e-13 * np.max(a["gabs"], initial=0))
