"""Shared helpers of the GPU parity tests: seeded inputs, the oracle side and
the tolerance gate.

Gate (per individual):  |f_gpu - f_ref| <= rtol * |f_ref| + atol * Var(y)
  float32 nodes: rtol = 1e-5, atol = 1e-10;  float64 nodes: rtol = 1e-12, atol = 1e-14.
Individuals the oracle's Monte-Carlo-arithmetic check flags as ill-conditioned
for the node precision are not held to the gate; for them the test checks
that the GPU result is a valid fitness (finite, 0 <= LS-MSE <= Var(y)) and
reports how many there were.  Status (non-finite / bad program) must match
exactly for every unflagged individual.
"""
import sys

import numpy as np

import paper_2605_30954_amd as gg
from oracle import fitness as OF, grad as OG, mca as OM, tree as OT
from synth import make_dataset, sample_population

GATE = {"f32": (1e-5, 1e-10), "f64": (1e-12, 1e-14)}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_inputs(cfg, M, N, salt=0):
    X, y = make_dataset(cfg, N=N, salt=salt)
    genes, gc, hs = sample_population(cfg, M=M, salt=salt)
    hv = hs if len(set(hs.tolist())) > 1 else int(hs[0])
    ops, cs, ln, nc = gg.encode(genes, gc, hv, cfg.L_max, cfg.C_max)  # the library's encoder
    return dict(cfg=cfg, X=X, y=y, genes=genes, gc=gc, hs=hs, ops=ops, cs=cs, ln=ln, nc=nc)


def to_device(d, device="cuda:0"):
    import torch
    return (torch.from_numpy(d["ops"]).to(device), torch.from_numpy(d["cs"]).to(device),
            torch.from_numpy(d["X"]).to(device), torch.from_numpy(d["y"]).to(device))


def oracle_scores(d, idx, linear_scaling=True, precision="f32"):
    return OF.evaluate_population(d["genes"], d["gc"], d["hs"], d["X"], d["y"],
                                  linear_scaling=linear_scaling, rng=precision, indices=idx)


def oracle_flags(d, idx, precision="f32", linear_scaling=True, with_grad=False, n=8):
    rtol = GATE[precision][0]
    return OM.flags(d["genes"], d["gc"], d["hs"], d["X"], d["y"], precision=precision, rtol=rtol,
                    linear_scaling=linear_scaling, with_grad=with_grad, indices=idx, n=n)


def gate_fitness(f_gpu, st_gpu, ref, flagged, vy, precision, what=""):
    """Assert the gate; return a report dict."""
    rtol, atol = GATE[precision]
    f_gpu = np.asarray(f_gpu, np.float64)
    st_gpu = np.asarray(st_gpu)
    fr = ref["fitness"]
    sr = ref["status"]
    errs, bad = [], []
    for q in range(len(fr)):
        if flagged[q]:
            if st_gpu[q] == 0:
                assert np.isfinite(f_gpu[q]) and f_gpu[q] >= 0, (what, q, f_gpu[q])
            continue
        assert st_gpu[q] == sr[q], (what, q, "status", int(st_gpu[q]), int(sr[q]))
        if sr[q] != 0:
            assert np.isinf(f_gpu[q])
            continue
        tol = rtol * abs(fr[q]) + atol * vy
        e = abs(f_gpu[q] - fr[q])
        errs.append(e / max(abs(fr[q]), 1e-300))
        if not e <= tol:   # a NaN fails too
            bad.append((q, f_gpu[q], fr[q], e / max(abs(fr[q]), 1e-300)))
    rep = dict(n=len(fr), flagged=int(np.sum(flagged)), gated=len(errs),
               max_rel=float(max(errs)) if errs else 0.0,
               median_rel=float(np.median(errs)) if errs else 0.0, failures=bad[:5])
    log(f"[parity] {what}: {rep}")
    assert not bad, f"{what}: {len(bad)} individuals outside the gate, e.g. {bad[:3]}"
    return rep


def oracle_gradients(d, idx, linear_scaling=True):
    out = []
    for m in idx:
        s, g = OG.gradient(d["genes"][m], d["gc"][m], int(d["hs"][m]), d["X"], d["y"],
                           linear_scaling=linear_scaling, rng="f32")
        out.append((s, g))
    return out


def partial_peak(d, m):
    """Largest |d p_r / d c_j| over rows and constants of individual m, float64
    (forward mode in the oracle): above the float32 range (3.4e38) a float32
    per-row partial overflows."""
    ev = OT.Evaluator(np.asarray(d["X"], np.float64), rng="f32", duals=True)
    p, dp = ev.run(d["genes"][m], d["gc"][m], int(d["hs"][m]))
    return float(np.max(np.abs(dp))) if dp.size else 0.0


# per-row partials and residuals are binary32: each term of the gradient's
# dot product carries a few unit roundoffs, so a cancelling sum is known only
# to about u32 * sum |terms| (the oracle's gabs)
U32 = 2.0 ** -24
GRAD_ROUND = 4.0 * U32


def gate_gradients(g_gpu, st_gpu, refs, flagged, vy, rtol=1e-5, atol=1e-10, what=""):
    """Normwise per individual:
    |g_gpu - g_ref|_inf <= rtol |g_ref|_inf + atol Var(y) + 4 u32 max_j gabs_j."""
    errs, bad = [], []
    for q, (s, g) in enumerate(refs):
        if flagged[q] or s["status"] != 0 or st_gpu[q] != 0:
            continue
        C = g.size
        gg_ = np.asarray(g_gpu[q][:C], np.float64)
        assert np.all(np.asarray(g_gpu[q][C:]) == 0), (what, q, "unused constants not zero")
        if C == 0:
            continue
        e = float(np.max(np.abs(gg_ - g)))
        sc = float(np.max(np.abs(g)))
        tol = rtol * sc + atol * vy + GRAD_ROUND * float(np.max(s["gabs"]))
        errs.append(e / max(sc, 1e-300))
        if not e <= tol:   # a NaN fails too
            bad.append((q, e, sc, tol))
    rep = dict(n=len(refs), flagged=int(np.sum(flagged)), gated=len(errs),
               max_rel=float(max(errs)) if errs else 0.0,
               median_rel=float(np.median(errs)) if errs else 0.0, failures=bad[:5])
    log(f"[parity-grad] {what}: {rep}")
    assert not bad, f"{what}: {len(bad)} gradients outside the gate, e.g. {bad[:3]}"
    return rep
