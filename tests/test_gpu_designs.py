"""The paper's two evaluation designs (Section 3.2, Fig. 2), kept as
comparators, through the C ABI: raw MSE (Eq. 1) against the oracle with the
parity gate on several workloads, against the fused path's raw MSE, across
block sizes and blocks per program (ragged row blocks, more blocks than rows),
and the status of bad and overflowing programs."""
import numpy as np
import pytest

import paper_2605_30954_amd as gg
from oracle import opset as O
from parity_util import gate_fitness, log, make_inputs, oracle_flags, oracle_scores, to_device
from synth import get_config

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cid,M,N", [(1, 64, 1000), (2, 128, 20011), (5, 48, 4099), (10, 32, 3001)])
def test_designs_match_the_oracle(cid, M, N):
    import dataclasses
    cfg = get_config(cid)
    if cid == 10:
        cfg = dataclasses.replace(cfg, heights=(8,))     # 511-token templates
    log(f"[case] designs cfg{cid} M={M} N={N}")
    d = make_inputs(cfg, M, N)
    ops, cs, X, y = to_device(d)
    idx = list(range(M))
    ref = oracle_scores(d, idx, linear_scaling=False)
    sens = oracle_flags(d, idx, "f32", linear_scaling=False, n=4)
    vy = float(np.var(d["y"].astype(np.float64)))
    fused = gg.eval_batch(ops, cs, X, y, linear_scaling=False).cpu().numpy()
    for design, block, nb in ((1, 256, 1), (1, 64, 1), (2, 256, 7), (2, 1024, 3)):
        f, st = gg.eval_design(ops, cs, X, y, design=design, block=block, blocks_per_program=nb,
                               return_status=True)
        f, st = f.cpu().numpy(), st.cpu().numpy()
        gate_fitness(f, st, ref, sens, vy, "f32", f"design {design} block {block} x {nb} cfg{cid}")
        ok = st == 0
        np.testing.assert_allclose(f[ok], fused[ok], rtol=1e-6, atol=1e-12 * vy)


def test_design2_more_blocks_than_rows():
    cfg = get_config(2)
    d = make_inputs(cfg, 16, 100)
    ops, cs, X, y = to_device(d)
    f1 = gg.eval_design(ops, cs, X, y, design=1, block=64).cpu().numpy()
    f2 = gg.eval_design(ops, cs, X, y, design=2, block=64, blocks_per_program=300).cpu().numpy()
    np.testing.assert_allclose(f2, f1, rtol=1e-12)


def test_design_status_of_bad_and_overflowing_programs():
    import torch
    C, V0, E = O.CONST, O.VAR0, -1
    L = 40
    progs = [
        ([V0, V0, O.ADD], []),                                   # fine
        ([C, O.ADD], [1.0]),                                     # stack underflow
        ([V0 + 5], []),                                          # variable >= F (F = 2)
        ([C, C, C, O.ADD, O.ADD], [1.0, 1.0]),                   # more constants than C_max = 2
        ([V0] * 17 + [O.ADD] * 16, []),                          # 17 operands: deeper than 16
        ([V0] * 16 + [O.ADD] * 15, []),                          # 16 operands: fine
        ([C, C, O.MUL], [1e30, 1e30]),                           # overflows binary32
        ([V0, V0], []),                                          # two results
        ([], []),                                                # empty
        ([44], []),                                              # unknown symbol
    ]
    ops = np.full((len(progs), L), E, dtype=np.int8)
    cs = np.zeros((len(progs), 2), dtype=np.float32)
    for i, (t, c) in enumerate(progs):
        ops[i, : len(t)] = t
        cs[i, : len(c)] = c
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (2, 777)).astype(np.float32)
    y = rng.uniform(-1, 1, 777).astype(np.float32)
    dv = lambda a: torch.from_numpy(a).to("cuda:0")
    want = [0, 2, 2, 2, 2, 0, 1, 2, 2, 2]
    for design in (1, 2):
        f, st = gg.eval_design(dv(ops), dv(cs), dv(X), dv(y), design=design, block=128,
                               blocks_per_program=5, return_status=True)
        f, st = f.cpu().numpy(), st.cpu().numpy()
        assert st.tolist() == want, (design, st.tolist())
        assert np.all(np.isinf(f[st != 0])) and np.all(np.isfinite(f[st == 0]))
        x0 = X[0].astype(np.float64)
        np.testing.assert_allclose(f[0], np.mean((2 * x0 - y) ** 2), rtol=1e-6)
        np.testing.assert_allclose(f[5], np.mean((16 * x0 - y) ** 2), rtol=1e-6)


def test_design_argument_errors():
    import torch
    ops = torch.full((2, 3), -1, dtype=torch.int8, device="cuda:0")
    cs = torch.zeros((2, 1), dtype=torch.float32, device="cuda:0")
    X = torch.zeros((1, 10), dtype=torch.float32, device="cuda:0")
    y = torch.zeros(10, dtype=torch.float32, device="cuda:0")
    for block in (32, 96, 2048):
        with pytest.raises(gg.LibraryError):
            gg.eval_design(ops, cs, X, y, design=1, block=block)
    with pytest.raises(gg.LibraryError):
        gg.eval_design(ops, cs, X, y, design=2, blocks_per_program=0)
