"""Constant optimisation on the device: the library's Adam step against the
binary64 reference (oracle/constopt.py), and Adam driven by the fused
fitness + gradient call recovering the constants of a generating formula."""
import numpy as np
import pytest

import paper_2605_30954_amd as gg
from oracle import constopt as OC
from oracle import opset as O
from paper_2605_30954_amd.constopt import adam_step, optimise_constants
from parity_util import log, make_inputs
from synth import get_config

pytestmark = pytest.mark.gpu


def test_adam_step_matches_reference():
    import torch
    rng = np.random.default_rng(4)
    M, C = 37, 70                  # C spans two strides of the 64 lanes, ragged
    c = rng.uniform(-3, 3, (M, C)).astype(np.float32)
    g = rng.standard_normal((M, C)) * 10.0 ** rng.uniform(-6, 2, (M, 1))
    g[3, 5] = np.inf
    g[4, 6] = np.nan
    g[:, 60:] = 0.0                # unused constants
    m1 = (rng.standard_normal((M, C)) * 0.1).astype(np.float32)
    m2 = (rng.uniform(0, 1, (M, C)) * 0.01).astype(np.float32)
    bc = rng.uniform(-3, 3, (M, C)).astype(np.float32)
    bf = rng.uniform(0.5, 1.5, M)
    bf[0] = np.inf
    f = rng.uniform(0, 2, M)
    f[[7, 8]] = np.inf
    f[9] = np.nan
    t, lr = 3, 0.05
    d = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dt)
    cd, mom = d(c, torch.float32), d(np.stack([m1, m2]), torch.float32)
    bcd, bfd = d(bc, torch.float32), d(bf, torch.float64)
    adam_step(cd, d(g, torch.float64), d(f, torch.float64), mom, bcd, bfd, t, lr)
    want = OC.adam_step(c, g, f, m1, m2, bc, bf, t, lr)
    got_c, got_m = cd.cpu().numpy(), mom.cpu().numpy()
    np.testing.assert_array_equal(bfd.cpu().numpy(), want[4])
    np.testing.assert_array_equal(bcd.cpu().numpy(), want[3].astype(np.float32))
    ulp = np.spacing(np.abs(want[0]).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(got_c - want[0]) <= 4 * ulp + lr * 1e-5), np.max(np.abs(got_c - want[0]))
    # the moments are sums of two terms that may cancel: binary32 rounding is
    # bounded by a few units of the terms' magnitudes
    gg_ = np.where(np.isfinite(g), g, 0.0)
    scale1 = 0.9 * np.abs(m1) + 0.1 * np.abs(gg_)
    scale2 = 0.999 * np.abs(m2) + 0.001 * gg_ ** 2
    assert np.all(np.abs(got_m[0] - want[1]) <= 4 * 2.0 ** -24 * scale1 + 1e-38)
    assert np.all(np.abs(got_m[1] - want[2]) <= 4 * 2.0 ** -24 * scale2 + 1e-38)


@pytest.mark.timeout(300)
def test_optimise_constants_recovers_the_generating_constants():
    """2.3 x0^2 - 0.7 x1 x4 + cos(1.9 x2) with its three constants moved by up
    to 15 %, next to random programs of the same workload: Adam on the
    fitness gradient brings the formula's NMSE down by orders of magnitude,
    and no program ends worse than it started."""
    import torch
    cfg = get_config(4)
    N = 50_000
    d = make_inputs(cfg, 48, N, salt=5)
    X, y = d["X"], d["y"]
    ops, cs = d["ops"].copy(), d["cs"].copy()
    V = [O.VAR0 + k for k in range(10)]
    t = [O.CONST, V[0], V[0], O.MUL, O.MUL, O.CONST, V[1], O.MUL, V[4], O.MUL, O.SUB,
         O.CONST, V[2], O.MUL, O.COS, O.ADD]
    rng = np.random.default_rng(9)
    n_f = 16
    ops[:n_f] = -1
    ops[:n_f, : len(t)] = t
    cs[:n_f] = 0
    cs[:n_f, :3] = np.array([2.3, 0.7, 1.9]) * rng.uniform(0.85, 1.15, (n_f, 3))
    dev = lambda a: torch.from_numpy(a).to("cuda:0")
    opsd, csd, Xd, yd = dev(ops), dev(cs), dev(X), dev(y)
    f0 = gg.eval_batch(opsd, csd, Xd, yd).cpu().numpy()
    best_c, best_f = optimise_constants(opsd, csd, Xd, yd, steps=200, lr=0.02)
    bf = best_f.cpu().numpy()
    vy = float(np.var(y.astype(np.float64)))
    log(f"[constopt] formula NMSE median {np.median(f0[:n_f]) / vy:.3e} -> {np.median(bf[:n_f]) / vy:.3e}; "
        f"random programs improved {int(np.sum(bf[n_f:] < f0[n_f:]))}/{48 - n_f}")
    ok = np.isfinite(f0)
    assert np.all(bf[ok] <= f0[ok] * (1 + 1e-9))      # (the start point is measured again)
    assert np.median(bf[:n_f]) < 1e-2 * np.median(f0[:n_f])
    assert np.all(bf[:n_f] / vy < 1e-3)
    # the kept fitness is the kept constants' fitness
    f_again = gg.eval_batch(opsd, best_c, Xd, yd).cpu().numpy()
    np.testing.assert_allclose(f_again[ok], bf[ok], rtol=1e-9, atol=1e-14 * vy)
