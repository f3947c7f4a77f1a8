"""The formula-ladder workloads (Tab. 1, Experiment III) on the device.

Each of Addition, Division, Subtraction, Multiplication and Squaring (Feynman
I.9.18) at its full size (100,000 rows x 9 features, operator set of Tab. 2),
with a population on depth-6 templates (127 nodes; 2,000 individuals, the
paper's smaller population) and on depth-8 templates (511 nodes, 512
individuals).  The generating expression is planted three times (first, middle
and last program, each with other introns) among random individuals and must
reach NMSE <= 1e-6, the paper's success threshold for these problems, with
binary32 nodes (and <= 1e-12 with binary64 nodes).  The whole batch goes
through the fused fitness + gradient path; a sample (the planted programs plus
random ones) is graded against the oracle with the parity gate, and every
program against the properties that hold at any size."""
import dataclasses

import numpy as np
import pytest

import paper_2605_30954_amd as gg
from oracle import fast
from parity_util import check_properties, gate_fitness, gate_gradients, log, to_device
from synth import LADDER, get_config, ladder, make_dataset, sample_population

pytestmark = pytest.mark.gpu

NMSE_SUCCESS = 1e-6


def _inputs(cid, height, M):
    cfg = dataclasses.replace(get_config(cid), heights=(height,))
    X, y = make_dataset(cfg)
    genes, gc, hs = sample_population(cfg, M=M)
    planted = [0, M // 2 + 1, M - 1]
    for q, m in enumerate(planted):
        genes[m], gc[m] = ladder.genotype(ladder.GENERATING[cid], height, cfg.F, cfg.funcs, seed=q)
    ops, cs, ln, nc = gg.encode(genes, gc, height, cfg.L_max, cfg.C_max)
    return dict(cfg=cfg, X=X, y=y, genes=genes, gc=gc, hs=hs, ops=ops, cs=cs, ln=ln, nc=nc,
                planted=planted)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("height,M", [(6, 2000), (8, 512)])
@pytest.mark.parametrize("cid", sorted(LADDER))
def test_ladder_generating_tree_and_parity(cid, height, M):
    import torch
    d = _inputs(cid, height, M)
    log(f"[case] ladder {d['cfg'].name} depth {height} M={M} N={d['cfg'].N}")
    ops, cs, X, y = to_device(d)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        fit, grad, aux, st = gg.grad_consts(ops, cs, X, y, return_aux=True, return_status=True)
        f64, aux64 = gg.eval_batch(ops, cs, X, y, fp64_nodes=True, return_aux=True)
    s.synchronize()
    fit, grad, aux, st = [t.cpu().numpy() for t in (fit, grad, aux, st)]
    aux64 = aux64.cpu().numpy()
    vy = float(np.var(d["y"].astype(np.float64)))
    check_properties(fit, aux, st, grad, d["nc"].astype(np.int64), vy)
    for m in d["planted"]:
        log(f"[nmse] program {m}: f32 nodes {aux[m, 3]:.3e}, f64 nodes {aux64[m, 3]:.3e}")
        assert st[m] == 0 and aux[m, 3] <= NMSE_SUCCESS
        assert aux64[m, 3] <= 1e-12
    rng = np.random.default_rng([cid, height])
    rest = np.setdiff1d(np.arange(M), d["planted"])
    idx = sorted(d["planted"] + rng.choice(rest, size=13, replace=False).tolist())
    sens = fast.sensitivity(d["genes"], d["gc"], d["hs"], d["X"], d["y"], n=3, with_grad=True,
                            indices=idx)
    refs = [fast.run(d["genes"][m], d["gc"][m], height, d["X"], d["y"], with_grad=True) for m in idx]
    ref = {k: np.array([r[k] for r in refs]) for k in ("fitness", "status")}
    rep = gate_fitness(fit[idx], st[idx], ref, sens, vy, "f32", f"ladder {cid} depth {height}")
    grep = gate_gradients(grad[idx], st[idx], [(r, r["grad"]) for r in refs], sens, vy,
                          what=f"ladder {cid} depth {height}")
    assert rep["gated"] == len(idx)
    assert grep["compared"] + grep["status_sensitive"] >= 4
