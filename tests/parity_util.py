"""Shared helpers of the GPU parity tests: seeded inputs, the oracle side and
the tolerance gate.

Gate (every individual is graded; none is skipped):
    |f_gpu - f_ref| <= rtol |f_ref| + atol Var(y) + K_SPREAD * spread
  float32 nodes: rtol = 1e-5, atol = 1e-10;  float64 nodes: rtol = 1e-12, atol = 1e-14.
``spread`` is the individual's own sensitivity to the node precision, measured
by the oracle (oracle/mca.py: Monte-Carlo arithmetic runs and runs with the
protection thresholds moved by 1e-4): the largest deviation of the fitness over
those runs.  A well-conditioned individual has a spread far below the first two
terms; an ill-conditioned one is still compared value by value, with the
tolerance its conditioning implies.  Where some run changes the status
(finite / not finite) the spread is infinite: either status is accepted and a
status-0 result must be a valid fitness (finite, 0 <= LS-MSE <= Var(y)).
Status must otherwise match exactly.

Gradients, normwise per individual:
    |g_gpu - g_ref|_inf <= rtol |g_ref|_inf + atol Var(y) + 4 u32 max_j gabs_j + K_SPREAD * gspread
with gabs the sum of the magnitudes of the gradient's per-row terms (the
binary32 per-row terms and per-lane binary32 sums of the device carry a few
unit roundoffs of it; Higham, Sec. 3.1) and gspread the oracle's measured
sensitivity of the gradient.
"""
import sys

import numpy as np

import paper_2605_30954_amd as gg
from oracle import fitness as OF, grad as OG, mca as OM, tree as OT
from synth import make_dataset, sample_population

GATE = {"f32": (1e-5, 1e-10), "f64": (1e-12, 1e-14)}
#: multiple of the measured sensitivity added to the gate: the spread is the
#: largest deviation over about ten runs that perturb every node by up to one
#: unit roundoff; the device's own rounding (transcendentals a few ulp) is of
#: that order, so three spreads bound it with margin
K_SPREAD = 3.0


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_inputs(cfg, M, N, salt=0):
    X, y = make_dataset(cfg, N=N, salt=salt)
    genes, gc, hs = sample_population(cfg, M=M, salt=salt)
    hv = hs if len(set(hs.tolist())) > 1 else int(hs[0])
    ops, cs, ln, nc = gg.encode(genes, gc, hv, cfg.L_max, cfg.C_max)  # the library's encoder
    return dict(cfg=cfg, X=X, y=y, genes=genes, gc=gc, hs=hs, ops=ops, cs=cs, ln=ln, nc=nc)


def check_properties(fit, aux, st, grad, nc, vy):
    """Properties of every individual's result that hold at any size: status 0
    exactly when the fitness is finite, 0 <= LS-MSE <= Var(y), NMSE =
    fitness / Var(y), a zero gradient past the last constant and for a
    non-finite individual."""
    ok = st == 0
    assert np.array_equal(np.isfinite(fit), ok)
    assert np.all(fit[ok] >= 0.0) and np.all(fit[ok] <= vy * (1 + 1e-9))
    np.testing.assert_allclose(aux[ok, 3], fit[ok] / vy, rtol=1e-12)   # Var(y) summed in another order
    if grad is not None:
        C = grad.shape[1]
        past = np.arange(C)[None, :] >= nc[:, None]
        assert np.all(grad[past] == 0.0)
        assert np.all(grad[~ok] == 0.0)


def to_device(d, device="cuda:0"):
    import torch
    return (torch.from_numpy(d["ops"]).to(device), torch.from_numpy(d["cs"]).to(device),
            torch.from_numpy(d["X"]).to(device), torch.from_numpy(d["y"]).to(device))


def oracle_scores(d, idx, linear_scaling=True, precision="f32"):
    return OF.evaluate_population(d["genes"], d["gc"], d["hs"], d["X"], d["y"],
                                  linear_scaling=linear_scaling, rng=precision, indices=idx)


def oracle_flags(d, idx, precision="f32", linear_scaling=True, with_grad=False, n=8):
    """Per-individual sensitivity (oracle/mca.py) of the listed individuals:
    the spreads that widen each one's tolerance."""
    return OM.sensitivity(d["genes"], d["gc"], d["hs"], d["X"], d["y"], precision=precision,
                          linear_scaling=linear_scaling, with_grad=with_grad, indices=idx, n=n)


def ill_mask(sens, f_ref, vy, precision="f32"):
    """True where an individual is ill-conditioned for the node precision
    (its spread exceeds a tenth of the plain gate, or a decision sits within
    the window of its threshold or flips)."""
    return np.array([_ill(s, f, vy, precision) for s, f in zip(sens, f_ref)], dtype=bool)


def _ill(s, f_ref, vy, precision):
    rtol, atol = GATE[precision]
    return bool(s["flipped"] or s["near"] or
                s["fit_spread"] > (rtol * abs(f_ref) + atol * vy) / 10)


def gate_fitness(f_gpu, st_gpu, ref, sens, vy, precision, what=""):
    """Assert the gate for every individual; return a report dict."""
    rtol, atol = GATE[precision]
    f_gpu = np.asarray(f_gpu, np.float64)
    st_gpu = np.asarray(st_gpu)
    fr = ref["fitness"]
    sr = ref["status"]
    errs, bad = [], []
    n_ill = n_loose = 0
    for q in range(len(fr)):
        s = sens[q]
        n_ill += _ill(s, fr[q], vy, precision)
        if not np.isfinite(s["fit_spread"]):   # the status itself is sensitive
            n_loose += 1
            if st_gpu[q] == 0:
                ok = np.isfinite(f_gpu[q]) and f_gpu[q] >= 0 and f_gpu[q] <= vy * (1 + 1e-9)
                if not ok:
                    bad.append((q, f_gpu[q], fr[q], "invalid"))
            continue
        if st_gpu[q] != sr[q]:
            bad.append((q, int(st_gpu[q]), int(sr[q]), "status"))
            continue
        if sr[q] != 0:
            if not np.isinf(f_gpu[q]):
                bad.append((q, f_gpu[q], fr[q], "not inf"))
            continue
        tol = rtol * abs(fr[q]) + atol * vy + K_SPREAD * s["fit_spread"]
        e = abs(f_gpu[q] - fr[q])
        errs.append(e / max(abs(fr[q]), 1e-300))
        if not e <= tol:   # a NaN fails too
            bad.append((q, f_gpu[q], fr[q], e / max(abs(fr[q]), 1e-300)))
    rep = dict(n=len(fr), gated=len(fr), ill_conditioned=int(n_ill), status_sensitive=int(n_loose),
               compared=len(errs), max_rel=float(max(errs)) if errs else 0.0,
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


def gate_gradients(g_gpu, st_gpu, refs, sens, vy, rtol=1e-5, atol=1e-10, what=""):
    """Normwise per individual (see the module docstring); every individual
    with status 0 on both sides is compared."""
    errs, bad = [], []
    n_ill = n_loose = 0
    for q, (s, g) in enumerate(refs):
        C = g.size
        assert np.all(np.asarray(g_gpu[q][C:]) == 0), (what, q, "unused constants not zero")
        if s["status"] != 0 or st_gpu[q] != 0:
            continue                      # statuses are gated with the fitness
        gs = sens[q]["grad_spread"]
        if gs is None or not np.isfinite(gs):
            n_loose += 1
            continue
        if C == 0:
            continue
        gg_ = np.asarray(g_gpu[q][:C], np.float64)
        e = float(np.max(np.abs(gg_ - g)))
        sc = float(np.max(np.abs(g)))
        base = rtol * sc + atol * vy + GRAD_ROUND * float(np.max(s["gabs"]))
        n_ill += gs > base / 10 or sens[q]["flipped"] or sens[q]["near"]
        tol = base + K_SPREAD * gs
        errs.append(e / max(sc, 1e-300))
        if not e <= tol:   # a NaN fails too
            bad.append((q, e, sc, tol))
    rep = dict(n=len(refs), compared=len(errs), ill_conditioned=int(n_ill),
               status_sensitive=int(n_loose), max_rel=float(max(errs)) if errs else 0.0,
               median_rel=float(np.median(errs)) if errs else 0.0, failures=bad[:5])
    log(f"[parity-grad] {what}: {rep}")
    assert not bad, f"{what}: {len(bad)} gradients outside the gate, e.g. {bad[:3]}"
    return rep
