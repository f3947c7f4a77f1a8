"""The oracle in C for workloads too large for NumPy (oracle/ctree.c).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test-suite
loads it.  It computes what tree.py, fitness.py, grad.py and mca.py compute,
from the same definitions, row by row in binary64 on several host threads,
and shares nothing with the HIP library.  tests/test_oracle_fast.py pins it to
the NumPy oracle (values, gradients, statuses, conditioning) on every workload.

Differences from the NumPy implementation, none of which changes a result
beyond binary64 rounding:
  * sums are Neumaier-compensated per thread, combined in thread order
    (NumPy: math.fsum / pairwise);
  * transcendental functions are the C library's (NumPy's own SIMD versions
    may differ by an ulp);
  * the Monte-Carlo perturbations come from a counter-based generator
    (splitmix64 of seed, slot and row) rather than NumPy's stream, and a
    decision counts as flipped when a status or the degenerate-fit case
    changes, or a threshold-shifted run changes the fitness (the NumPy
    version also compares every node's decisions between runs).
"""
import ctypes
import os
import subprocess

import numpy as np

from . import fitness as FT
from . import mca as MC
from . import opset as O

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "ctree.c")
LIB = os.path.join(_HERE, "libctree.so")


def build():
    """Compile ctree.c with the host C compiler (gcc)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        f = L.gg_oracle_run
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                      ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                      ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        _lib = L
    return _lib


def threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def run(genes_row, gconst_row, height, X, y, linear_scaling=True, rng="f32", thresholds=None,
        degenerate_rtol=FT.DEGENERATE_RTOL, eps=0.0, seed=0, window=1e-4, with_grad=True,
        return_p=False, nthreads=None):
    """Score dict (fitness, a, b, mse, nmse, status, vp, pbar, near) of one
    genotype; with_grad adds grad [C] and gabs [C]; return_p the predictions."""
    g = np.ascontiguousarray(genes_row, dtype=np.int8)
    gc = np.ascontiguousarray(np.asarray(gconst_row, dtype=np.float32), dtype=np.float64)
    X32 = np.ascontiguousarray(X, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    N = y32.size
    out = np.zeros(10 + 2 * 256, dtype=np.float64)
    p = np.empty(N, dtype=np.float64) if return_p else None
    guard, clamp = thresholds if thresholds else (0.0, 0.0)
    nc = lib().gg_oracle_run(g.ctypes.data, gc.ctypes.data, g.size, int(height), X32.ctypes.data, N,
                             y32.ctypes.data, int(bool(linear_scaling)), int(rng == "f32"), float(guard),
                             float(clamp), float(degenerate_rtol), float(eps), int(seed) & (2 ** 64 - 1),
                             float(window), int(bool(with_grad)), int(nthreads or threads()),
                             out.ctypes.data, p.ctypes.data if p is not None else None)
    if nc < 0:
        raise ValueError("malformed genotype or too many constants")
    s = dict(fitness=out[0], a=out[1], b=out[2], mse=out[3], nmse=out[4], status=int(out[5]),
             near=bool(out[6]), vp=out[8], pbar=out[9])
    if with_grad:
        s["grad"] = out[10:10 + nc].copy()
        s["gabs"] = out[10 + nc:10 + 2 * nc].copy()
    if return_p:
        s["p"] = p
    return s


def gradient(genes_row, gconst_row, height, X, y, linear_scaling=True, rng="f32"):
    """(score dict with gabs, grad[C]) like oracle.grad.gradient."""
    s = run(genes_row, gconst_row, height, X, y, linear_scaling, rng)
    return s, s["grad"]


def evaluate_population(genes, gconst, heights, X, y, linear_scaling=True, rng="f32", indices=None):
    M = genes.shape[0]
    hs = np.broadcast_to(np.asarray(heights), (M,))
    idx = range(M) if indices is None else indices
    out = {k: [] for k in ("fitness", "a", "b", "mse", "nmse", "status")}
    for m in idx:
        s = run(genes[m], gconst[m], int(hs[m]), X, y, linear_scaling, rng, with_grad=False)
        for k in out:
            out[k].append(s[k])
    return {k: np.asarray(v) for k, v in out.items()}


def sensitivity(genes, gconst, heights, X, y, precision="f32", n=8, seed=0, linear_scaling=True,
                window=1e-4, with_grad=False, indices=None):
    """Same contract as oracle.mca.sensitivity; each dict also holds "ref",
    the unperturbed run's result (score, and grad / gabs with with_grad)."""
    M = genes.shape[0]
    hs = np.broadcast_to(np.asarray(heights), (M,))
    idx = list(range(M)) if indices is None else list(indices)
    eps = MC.EPS[precision]
    res = []
    for m in idx:
        h = int(hs[m])
        s0 = run(genes[m], gconst[m], h, X, y, linear_scaling, precision, window=window, with_grad=with_grad)
        info = dict(fitness=s0["fitness"], status=s0["status"], fit_spread=0.0,
                    grad_spread=0.0 if with_grad else None, flipped=False, near=s0["near"], ref=s0)
        if s0["status"] == 0 and 0 < s0["vp"] <= 1e2 * FT.DEGENERATE_RTOL * max(s0["pbar"] ** 2, 1e-300):
            info["near"] = True
        runs = [("mca", k) for k in range(n)] + [("shift", +1), ("shift", -1)]
        for kind, k in runs:
            if kind == "mca":
                sk = run(genes[m], gconst[m], h, X, y, linear_scaling, precision, eps=eps,
                         seed=(seed * 1000003 + m) * 64 + k, window=window, with_grad=with_grad)
            else:
                thr = (O.GUARD * (1 + k * window), O.CLAMP * (1 - k * window))
                drt = FT.DEGENERATE_RTOL * (1e2 if k > 0 else 1e-2)
                sk = run(genes[m], gconst[m], h, X, y, linear_scaling, precision, thresholds=thr,
                         degenerate_rtol=drt, window=window, with_grad=with_grad)
            if sk["status"] != s0["status"]:
                info["flipped"] = True
                info["fit_spread"] = np.inf
                if with_grad:
                    info["grad_spread"] = np.inf
                continue
            if s0["status"] != 0:
                continue
            if (s0["b"] == 0.0) != (sk["b"] == 0.0) or (kind == "shift" and sk["fitness"] != s0["fitness"]):
                info["flipped"] = True
            info["fit_spread"] = max(info["fit_spread"], abs(sk["fitness"] - s0["fitness"]))
            if with_grad and s0["grad"].size:
                info["grad_spread"] = max(info["grad_spread"], float(np.max(np.abs(sk["grad"] - s0["grad"]))))
        res.append(info)
    return res
