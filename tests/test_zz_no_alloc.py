"""The no-allocation entry point (gpgomea_eval_batch_noalloc) against
gpgomea_eval_batch, through the C ABI: two calls in a row on one stream, the
second with fewer programs and rows; the results equal the workspace entry
point's bitwise (same kernels, same launch plan), both fitness kinds and the
plain form; a shape beyond the static scratch is refused with E_WORKSPACE."""
import ctypes

import numpy as np
import pytest

import paper_2605_30954_amd as gg
from paper_2605_30954_amd import _lib
from parity_util import log, make_inputs, to_device
from synth import get_config

pytestmark = pytest.mark.gpu


def _noalloc(ops, cs, X, y, flags, stream):
    import torch
    M, L = ops.shape
    C = cs.shape[1]
    F, N = X.shape
    fit = torch.full((M,), -1.0, dtype=torch.float64, device=ops.device)
    aux = torch.full((M, 4), -1.0, dtype=torch.float64, device=ops.device)
    st = torch.full((M,), -1, dtype=torch.int8, device=ops.device)
    rc = _lib.lib.gpgomea_eval_batch_noalloc(
        ops.data_ptr(), M, L, cs.data_ptr() if C else None, C, X.data_ptr(), F, N, N, y.data_ptr(),
        flags, fit.data_ptr(), aux.data_ptr(), st.data_ptr(), ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, _lib.last_error()
    return fit, aux, st


def test_noalloc_matches_workspace_entry_point():
    import torch
    cfg = get_config(4)
    d = make_inputs(cfg, 256, 20011, salt=3)
    ops, cs, X, y = to_device(d)
    s = torch.cuda.Stream()
    cases = [(256, 20011), (37, 3001)]   # the second call is smaller
    for ls in (True, False):
        for plain in (False, True):
            flags = gg.flags_of(ls, False, plain, graph=False)
            for M, N in cases:
                o, c = ops[:M].contiguous(), cs[:M].contiguous()
                Xs, ys = X[:, :N].contiguous(), y[:N].contiguous()
                log(f"[case] noalloc M={M} N={N} ls={ls} plain={plain}")
                with torch.cuda.stream(s):
                    f1, a1, s1 = _noalloc(o, c, Xs, ys, flags, s)
                    f2, a2, s2 = gg.eval_batch(o, c, Xs, ys, linear_scaling=ls, plain=plain, graph=False,
                                               return_aux=True, return_status=True)
                s.synchronize()
                assert torch.equal(s1, s2)
                assert np.array_equal(f1.cpu().numpy(), f2.cpu().numpy(), equal_nan=True)
                assert np.array_equal(a1.cpu().numpy(), a2.cpu().numpy(), equal_nan=True)


def test_noalloc_refuses_shapes_beyond_its_scratch():
    import torch
    cap = int(_lib.lib.gpgomea_noalloc_scratch_bytes())
    assert cap == 64 << 20
    M = 8192   # forward partials alone: 8192 x 256 spans x 32 B > 64 MiB
    ops = torch.full((M, 255), -1, dtype=torch.int8, device="cuda:0")
    ops[:, 0] = 64
    cs = torch.zeros((M, 1), dtype=torch.float32, device="cuda:0")
    X = torch.ones((1, 1000), dtype=torch.float32, device="cuda:0")
    y = torch.ones(1000, dtype=torch.float32, device="cuda:0")
    fit = torch.empty(M, dtype=torch.float64, device="cuda:0")
    rc = _lib.lib.gpgomea_eval_batch_noalloc(ops.data_ptr(), M, 255, cs.data_ptr(), 1, X.data_ptr(), 1,
                                             1000, 1000, y.data_ptr(), 1, fit.data_ptr(), None, None,
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _lib.E_WORKSPACE, rc
    assert "no-allocation" in _lib.last_error()
