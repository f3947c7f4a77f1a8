"""Batched GP-GOMEA fitness and constant-gradient evaluation on MI355X (gfx950).

Python face of libgpgomea_eval.so (see include/gpgomea_eval.h): it passes
torch device pointers and the current HIP stream to the C ABI and returns
torch tensors.  torch supplies device memory and streams only; every step of
the evaluation runs in the library's HIP kernels.

    fitness = eval_batch(ops, consts, X, y)                   # LS-MSE per program
    fitness, grad = grad_consts(ops, consts, X, y)            # + d fitness / d consts
    ops, consts, lens, nconst = encode(genes, gene_consts, heights, L_max, C_max)
"""
import ctypes
import os

import numpy as np

from . import _lib
from ._lib import (LINEAR_SCALING, FP64_NODES, PLAIN, NO_GRAPH, LibraryError,  # noqa: F401
                   MAX_LEN, MAX_CONSTS, MAX_FEATURES, check, last_error, lib)

#: launch shapes chosen by the autotuner on MI355X for the workloads of this
#: repository (load with load_tuning(); the library never reads it by itself)
TUNING_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "mi355x.json")

__all__ = ["eval_batch", "eval_batch_noalloc", "eval_design", "grad_consts", "encode", "decode", "validate", "workspace_bytes",
           "autotune", "load_tuning", "clear_graphs", "graph_count", "flags_of", "profile",
           "profile_report", "op_costs", "GPGOMEAFitness", "LibraryError"]


def _torch():
    import torch
    return torch


def flags_of(linear_scaling=True, fp64_nodes=False, plain=False, graph=True) -> int:
    f = 0
    if linear_scaling:
        f |= LINEAR_SCALING
    if fp64_nodes:
        f |= FP64_NODES
    if plain:
        f |= PLAIN
    if not graph:
        f |= NO_GRAPH
    return f


def workspace_bytes(M, L_max, C_max, F, N, flags) -> int:
    n = lib.gpgomea_workspace_bytes(int(M), int(L_max), int(C_max), int(F), int(N), int(flags))
    if n == 0:
        raise LibraryError(_lib.E_SHAPE, last_error())
    return int(n)


_WS = {}


def _workspace(device, stream, nbytes):
    """A cached uint8 device buffer per (device, stream), grown on demand
    (256-aligned: the caching allocator hands out 512-byte aligned blocks).
    It is allocated while ``stream`` is current, so the caching allocator ties
    it to that stream: when it is replaced by a larger one, its memory is
    reused only by work ordered after the calls that used it.  One workspace
    serves one stream; calls on one stream never overlap."""
    torch = _torch()
    key = (str(device), int(stream.cuda_stream))
    buf = _WS.get(key)
    if buf is None or buf.numel() < nbytes:
        with torch.cuda.stream(stream):
            buf = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=device)
        _WS[key] = buf
    return buf


def _dev_tensor(t, dtype, name, device=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on a GPU")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU (this library has no CPU path)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t.contiguous()


def _prep(ops, consts, X, y):
    torch = _torch()
    ops = _dev_tensor(ops, torch.int8, "ops")
    dev = ops.device
    consts = _dev_tensor(consts, torch.float32, "consts", dev)
    X = _dev_tensor(X, torch.float32, "X", dev)
    y = _dev_tensor(y, torch.float32, "y", dev)
    if ops.dim() != 2 or consts.dim() != 2 or X.dim() != 2 or y.dim() != 1:
        raise ValueError("expected ops [M, L], consts [M, C], X [F, N], y [N]")
    M, L = ops.shape
    if consts.shape[0] != M:
        raise ValueError("ops and consts disagree on M")
    F, N = X.shape
    if y.shape[0] != N:
        raise ValueError("X and y disagree on N")
    return ops, consts, X, y, dev, int(M), int(L), int(consts.shape[1]), int(F), int(N)


def _stream(dev):
    return _torch().cuda.current_stream(dev)


def eval_batch(ops, consts, X, y, linear_scaling=True, fp64_nodes=False, plain=False,
               graph=True, return_aux=False, return_status=False):
    """Fitness (float64 [M]) of M postfix programs on X (float32 [F, N],
    feature-major) and y (float32 [N]).  ``return_aux`` adds a [M, 4] tensor
    (a, b, MSE, NMSE); ``return_status`` adds int8 [M] (0 ok, 1 non-finite,
    2 bad program)."""
    torch = _torch()
    ops, consts, X, y, dev, M, L, C, F, N = _prep(ops, consts, X, y)
    flags = flags_of(linear_scaling, fp64_nodes, plain, graph)
    fit = torch.empty(M, dtype=torch.float64, device=dev)
    aux = torch.empty((M, 4), dtype=torch.float64, device=dev) if return_aux else None
    st = torch.empty(M, dtype=torch.int8, device=dev)
    s = _stream(dev)
    ws = _workspace(dev, s, workspace_bytes(M, L, C, F, N, flags))
    check(lib.gpgomea_eval_batch(
        ops.data_ptr(), M, L, consts.data_ptr() if C else None, C, X.data_ptr(), F, N, N,
        y.data_ptr(), flags, fit.data_ptr(), aux.data_ptr() if aux is not None else None,
        st.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.c_void_p(s.cuda_stream)))
    out = [fit]
    if return_aux:
        out.append(aux)
    if return_status:
        out.append(st)
    return out[0] if len(out) == 1 else tuple(out)


def eval_batch_noalloc(ops, consts, X, y, fitness, status=None, aux=None, linear_scaling=True,
                       fp64_nodes=False, plain=False):
    """gpgomea_eval_batch_noalloc: fitness into the caller's ``fitness``
    (float64 [M]; ``status`` int8 [M] and ``aux`` float64 [M, 4] optional), with
    the library's static scratch: the call allocates nothing (the outputs are
    the caller's)."""
    torch = _torch()
    ops, consts, X, y, dev, M, L, C, F, N = _prep(ops, consts, X, y)
    fitness = _dev_tensor(fitness, torch.float64, "fitness", dev)
    if status is not None:
        status = _dev_tensor(status, torch.int8, "status", dev)
    if aux is not None:
        aux = _dev_tensor(aux, torch.float64, "aux", dev)
    flags = flags_of(linear_scaling, fp64_nodes, plain, graph=False)
    check(lib.gpgomea_eval_batch_noalloc(
        ops.data_ptr(), M, L, consts.data_ptr() if C else None, C, X.data_ptr(), F, N, N,
        y.data_ptr(), flags, fitness.data_ptr(), aux.data_ptr() if aux is not None else None,
        status.data_ptr() if status is not None else None,
        ctypes.c_void_p(_stream(dev).cuda_stream)))
    return fitness


def eval_design(ops, consts, X, y, design=1, block=256, blocks_per_program=16,
                return_status=False):
    """Raw MSE (float64 [M]) with one of the paper's two evaluation designs
    (gpgomea_eval_design1 / gpgomea_eval_design2): the comparators of the
    fused path.  ``block`` threads per workgroup; design 2 uses
    ``blocks_per_program`` workgroups per program."""
    torch = _torch()
    ops, consts, X, y, dev, M, L, C, F, N = _prep(ops, consts, X, y)
    fit = torch.empty(M, dtype=torch.float64, device=dev)
    st = torch.empty(M, dtype=torch.int8, device=dev)
    s = ctypes.c_void_p(_stream(dev).cuda_stream)
    args = (ops.data_ptr(), M, L, consts.data_ptr() if C else None, C, X.data_ptr(), F, N, N,
            y.data_ptr(), int(block))
    if design == 1:
        check(lib.gpgomea_eval_design1(*args, fit.data_ptr(), st.data_ptr(), s))
    elif design == 2:
        part = torch.empty(max(1, M * int(blocks_per_program)), dtype=torch.float64, device=dev)
        check(lib.gpgomea_eval_design2(*args, int(blocks_per_program), part.data_ptr(), fit.data_ptr(),
                                       st.data_ptr(), s))
    else:
        raise ValueError("design must be 1 or 2")
    return (fit, st) if return_status else fit


def grad_consts(ops, consts, X, y, linear_scaling=True, plain=False, graph=True,
                return_aux=False, return_status=False):
    """(fitness [M], grad [M, C]) in float64: the gradient of each fitness with
    respect to that program's constants (zero past its last constant)."""
    torch = _torch()
    ops, consts, X, y, dev, M, L, C, F, N = _prep(ops, consts, X, y)
    flags = flags_of(linear_scaling, False, plain, graph)
    fit = torch.empty(M, dtype=torch.float64, device=dev)
    grad = torch.empty((M, C), dtype=torch.float64, device=dev)
    aux = torch.empty((M, 4), dtype=torch.float64, device=dev) if return_aux else None
    st = torch.empty(M, dtype=torch.int8, device=dev)
    s = _stream(dev)
    ws = _workspace(dev, s, workspace_bytes(M, L, C, F, N, flags))
    check(lib.gpgomea_grad_consts(
        ops.data_ptr(), M, L, consts.data_ptr() if C else None, C, X.data_ptr(), F, N, N,
        y.data_ptr(), flags, fit.data_ptr(), aux.data_ptr() if aux is not None else None,
        grad.data_ptr() if C else None, st.data_ptr(), ws.data_ptr(), ws.numel(),
        ctypes.c_void_p(s.cuda_stream)))
    out = [fit, grad]
    if return_aux:
        out.append(aux)
    if return_status:
        out.append(st)
    return tuple(out)


def autotune(ops, consts, X, y, linear_scaling=True, with_grad=False, cache_path=None, trials=3,
             fp64_nodes=False):
    """Time the fused kernels' launch parameters (rows per lane, rows per LDS
    tile, individuals per block) on these inputs and keep the fastest for this
    problem class in the process; with ``cache_path`` also merge the choice
    into that file.  Synchronises the current stream.  Returns the library's
    one-line description of the choice."""
    ops, consts, X, y, dev, M, L, C, F, N = _prep(ops, consts, X, y)
    flags = flags_of(linear_scaling, fp64_nodes)
    s = _stream(dev)
    ws = _workspace(dev, s, workspace_bytes(M, L, C, F, N, flags))
    desc = ctypes.create_string_buffer(512)
    check(lib.gpgomea_autotune(
        ops.data_ptr(), M, L, consts.data_ptr() if C else None, C, X.data_ptr(), F, N, N,
        y.data_ptr(), flags, int(bool(with_grad)), ws.data_ptr(), ws.numel(),
        cache_path.encode() if cache_path else None, int(trials), desc, 512,
        ctypes.c_void_p(s.cuda_stream)))
    return desc.value.decode()


def load_tuning(cache_path=TUNING_FILE):
    """Load a tuning file written by autotune (by default the shipped MI355X
    one); returns the number of entries."""
    n = lib.gpgomea_load_tuning(str(cache_path).encode())
    if n < 0:
        raise LibraryError(n, last_error())
    return n


def clear_graphs():
    check(lib.gpgomea_clear_graphs())


def graph_count() -> int:
    """Number of executable graphs the library holds (at most 16)."""
    return int(lib.gpgomea_graph_count())


def profile(enable: bool):
    """Bracket every kernel of later calls with hipEvents (graphs bypassed)."""
    check(lib.gpgomea_profile(int(bool(enable))))


def profile_report() -> dict:
    """{kernel kind: (launches, total_ms)} since the previous report."""
    n = lib.gpgomea_profile_report(None, 0)
    buf = ctypes.create_string_buffer(max(n, 1))
    check(lib.gpgomea_profile_report(buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def op_costs(iters=2048, device="cuda:0"):
    """Measured seconds per lane-application of every operator (see
    gpgomea_op_costs); keys are operator names."""
    torch = _torch()
    scratch = torch.empty(2048, dtype=torch.float32, device=device)
    out = (ctypes.c_double * 17)()
    check(lib.gpgomea_op_costs(out, 17, int(iters), scratch.data_ptr(),
                               ctypes.c_void_p(_stream(scratch.device).cuda_stream)))
    names = {1: "add", 2: "sub", 3: "rsub", 4: "mul", 5: "div", 6: "rdiv", 7: "pow", 8: "rpow",
             9: "sin", 10: "cos", 11: "sq", 12: "sqrt", 13: "exp", 14: "log", 16: "moments"}
    return {v: out[k] for k, v in names.items()}


# ------------------------------------------------------------- host codec
def _np(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def encode(genes, gene_consts, heights, L_max, C_max):
    """Genotypes (int8 [M, T] heap order, float32 [M, T]) -> postfix programs.
    ``heights`` is an int or int8 [M].  Returns (ops int8 [M, L_max],
    consts float32 [M, C_max], len int16 [M], nconst int16 [M])."""
    g = _np(genes, np.int8)
    c = _np(gene_consts, np.float32)
    M, T = g.shape
    hs = None
    h0 = 0
    if np.ndim(heights) == 0:
        h0 = int(heights)
    else:
        hs = _np(heights, np.int8)
    ops = np.empty((M, L_max), np.int8)
    cs = np.empty((M, C_max), np.float32)
    ln = np.empty(M, np.int16)
    nc = np.empty(M, np.int16)
    bad = ctypes.c_int32(-1)
    rc = lib.gpgomea_encode(g.ctypes.data, c.ctypes.data, M, T, h0,
                            hs.ctypes.data if hs is not None else None, ops.ctypes.data, L_max,
                            cs.ctypes.data, C_max, ln.ctypes.data, nc.ctypes.data,
                            ctypes.byref(bad))
    if rc < 0:
        raise LibraryError(rc, f"{last_error()} (individual {bad.value})")
    return ops, cs, ln, nc


def decode(ops, consts, height):
    o = _np(ops, np.int8)
    c = _np(consts, np.float32)
    M, L = o.shape
    T = 2 ** (height + 1) - 1
    g = np.empty((M, T), np.int8)
    gc = np.empty((M, T), np.float32)
    bad = ctypes.c_int32(-1)
    rc = lib.gpgomea_decode(o.ctypes.data, c.ctypes.data, M, L, c.shape[1], int(height),
                            g.ctypes.data, gc.ctypes.data, ctypes.byref(bad))
    if rc < 0:
        raise LibraryError(rc, f"{last_error()} (individual {bad.value})")
    return g, gc


def validate(ops, C_max, F, max_height=-1, return_first_bad=False):
    o = _np(ops, np.int8)
    M, L = o.shape
    st = np.empty(M, np.int8)
    first = ctypes.c_int32(-1)
    check(lib.gpgomea_validate(o.ctypes.data, M, L, int(C_max), int(F), int(max_height),
                               st.ctypes.data, ctypes.byref(first)))
    return (st, first.value) if return_first_bad else st


from .autograd import GPGOMEAFitness  # noqa: E402
