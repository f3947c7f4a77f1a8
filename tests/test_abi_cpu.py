"""C ABI checks that need no GPU: exported symbols, the host codec against the
oracle's codec (byte-exact), validation, and errors detected before launch."""
import ctypes
import json
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2605_30954_amd as gg
from paper_2605_30954_amd import _lib
from oracle import codec as OC, opset as O
from synth import CONFIGS, get_config, sample_population
from test_oracle_codec import all_height2_genotypes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpgomea_eval.h")
OPS_H = os.path.join(ROOT, "include", "gpgomea_ops.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gpgomea_\w+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (gpgomea_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(names) == set(_lib.SIGNATURES)
    assert gg.lib.gpgomea_version() >= 10000


def test_header_alphabet_matches_oracle_reading():
    txt = open(OPS_H).read()
    d = dict(re.findall(r"#define (GPGOMEA_\w+)\s+\(?(-?[0-9.e+-]+)\)?", txt))
    assert int(d["GPGOMEA_SYM_ADD"]) == O.ADD and int(d["GPGOMEA_SYM_SIN"]) == O.SIN
    assert int(d["GPGOMEA_SYM_POW"]) == O.POW and int(d["GPGOMEA_SYM_CONST"]) == O.CONST
    assert int(d["GPGOMEA_SYM_VAR0"]) == O.VAR0 and int(d["GPGOMEA_SYM_END"]) == O.END
    assert float(d["GPGOMEA_GUARD"]) == O.GUARD and float(d["GPGOMEA_CLAMP"]) == O.CLAMP


def test_fig1_library_encoding():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "fig1_example.json")))
    genes = np.array([g["genes"]], np.int8)
    gc = np.array([g["gene_consts"]], np.float32)
    ops, cs, ln, nc = gg.encode(genes, gc, 3, 15, 8)
    assert ops[0, : ln[0]].tolist() == g["expected_ops"]
    assert cs[0, : nc[0]].tolist() == g["expected_consts"]


def _same_encoding(genes, gc, heights, L, C):
    a = gg.encode(genes, gc, heights, L, C)
    b = OC.encode(genes, gc, heights, L, C)
    assert (a[0] == b[0]).all()
    assert (a[1].view(np.uint32) == b[1].view(np.uint32)).all()  # constant bit patterns
    assert (a[2] == b[2]).all() and (a[3] == b[3]).all()
    return a


def test_exhaustive_height2_library_vs_oracle():
    genes, gc = all_height2_genotypes()
    ops, cs, ln, nc = _same_encoding(genes, gc, 2, 7, 4)
    dg, dc = gg.decode(ops, cs, 2)
    og, oc = OC.decode(ops, cs, 2)
    assert (dg == og).all() and (dc.view(np.uint32) == oc.view(np.uint32)).all()


def test_exhaustive_height2_validate_heights():
    """validate's height check against the genotype: a program is taller than
    h exactly when one of its active slots lies below depth h of the template
    (Section 3.1's fixed template; depth from the heap index)."""
    from oracle.tree import active_slots, depth_of
    genes, gc = all_height2_genotypes()
    ops, cs, ln, nc = gg.encode(genes, gc, 2, 7, 4)
    depth = np.array([max(depth_of(s) for s in active_slots(g, 2)) for g in genes])
    assert set(depth.tolist()) == {0, 1, 2}
    for h in (-1, 0, 1, 2, 3):
        st, first = gg.validate(ops, 4, 2, max_height=h, return_first_bad=True)
        want = np.zeros(len(genes), np.int8) if h < 0 else np.where(depth > h, 2, 0).astype(np.int8)
        assert (st == want).all()
        bad = np.flatnonzero(want)
        assert first == (int(bad[0]) if len(bad) else -1)


@pytest.mark.parametrize("cid", sorted(CONFIGS))
def test_workload_populations_library_vs_oracle(cid):
    cfg = get_config(cid)
    genes, gc, hs = sample_population(cfg, M=min(cfg.M, 300), salt=11)
    hv = hs if len(set(hs.tolist())) > 1 else int(hs[0])
    ops, cs, ln, nc = _same_encoding(genes, gc, hv, cfg.L_max, cfg.C_max)
    dg, dc = gg.decode(ops, cs, cfg.h_max)
    og, oc = OC.decode(ops, cs, cfg.h_max)
    assert (dg == og).all() and (dc.view(np.uint32) == oc.view(np.uint32)).all()
    assert (gg.validate(ops, cfg.C_max, cfg.F) == 0).all()


def test_encode_errors():
    g = np.full((1, 7), O.VAR0, np.int8)
    g[0, 0] = O.ADD
    g[0, 1] = O.MUL           # operator whose children are the leaf slots 3 and 4: fine
    g[0, 3] = O.SIN           # active operator at a leaf slot: rejected
    with pytest.raises(gg.LibraryError) as e:
        gg.encode(g, np.zeros((1, 7), np.float32), 2, 7, 4)
    assert e.value.code == _lib.E_PROGRAM
    g[0, 3] = O.VAR0
    with pytest.raises(gg.LibraryError):       # does not fit L_max = 3
        gg.encode(g, np.zeros((1, 7), np.float32), 2, 3, 4)
    g[0, 3] = 17                               # unknown active symbol
    with pytest.raises(gg.LibraryError):
        gg.encode(g, np.zeros((1, 7), np.float32), 2, 7, 4)


def test_validate_statuses():
    progs = [
        [O.VAR0, O.VAR0 + 1, O.ADD],          # ok
        [O.ADD],                              # underflow
        [O.VAR0, O.VAR0],                     # two results
        [O.VAR0 + 5],                         # variable >= F (F=2)
        [O.CONST, O.CONST, O.MUL, O.CONST, O.ADD],  # 3 constants > C_max=2
        [17],                                 # unknown symbol
        [],                                   # empty
        [O.CONST, O.SIN],                     # ok
    ]
    ops = np.full((len(progs), 8), -1, np.int8)
    for i, p in enumerate(progs):
        ops[i, : len(p)] = p
    st = gg.validate(ops, 2, 2)
    assert st.tolist() == [0, 2, 2, 2, 2, 2, 2, 0]
    # heights of the two valid programs: 1 and 1
    st, first = gg.validate(ops, 2, 2, max_height=1, return_first_bad=True)
    assert st.tolist() == [0, 2, 2, 2, 2, 2, 2, 0] and first == 1
    st, first = gg.validate(ops, 2, 2, max_height=0, return_first_bad=True)
    assert st.tolist() == [2] * 8 and first == 0
    ok = ops[[0, 7]]
    st, first = gg.validate(ok, 2, 2, max_height=0, return_first_bad=True)
    assert st.tolist() == [2, 2] and first == 0
    st, first = gg.validate(ok, 2, 2, max_height=1, return_first_bad=True)
    assert st.tolist() == [0, 0] and first == -1
    # NULL status array: only the count and the first index
    f = ctypes.c_int32(7)
    assert gg.lib.gpgomea_validate(ops.ctypes.data, 8, 8, 2, 2, -1, None, ctypes.byref(f)) == 6
    assert f.value == 1
    with pytest.raises(gg.LibraryError):
        gg.validate(ops, 2, 2, max_height=-2)


def test_host_side_argument_errors():
    L = gg.lib
    fake = ctypes.c_void_p(256)
    ws_need = gg.workspace_bytes(4, 15, 8, 2, 1000, gg.LINEAR_SCALING)
    assert ws_need > 0

    def call(**kw):
        a = dict(ops=fake, M=4, L=15, consts=fake, C=8, X=fake, F=2, N=1000, ldx=1000, y=fake,
                 flags=gg.LINEAR_SCALING, fit=fake, aux=None, st=None, ws=fake, wsb=ws_need)
        a.update(kw)
        return L.gpgomea_eval_batch(a["ops"], a["M"], a["L"], a["consts"], a["C"], a["X"], a["F"],
                                    a["N"], a["ldx"], a["y"], a["flags"], a["fit"], a["aux"],
                                    a["st"], a["ws"], a["wsb"], None)
    assert call(ops=None) == _lib.E_ARG
    assert call(flags=0x100) == _lib.E_ARG
    assert call(M=0) == _lib.E_SHAPE
    assert call(L=600) == _lib.E_SHAPE
    assert call(F=0) == _lib.E_SHAPE
    assert call(N=0) == _lib.E_SHAPE
    assert call(ldx=999) == _lib.E_SHAPE
    assert call(wsb=ws_need - 1) == _lib.E_WORKSPACE
    assert call(ws=ctypes.c_void_p(256 + 8)) == _lib.E_WORKSPACE
    assert "workspace" in gg.last_error()
    assert L.gpgomea_workspace_bytes(0, 15, 8, 2, 1000, 1) == 0
    # the gradient entry point refuses binary64 nodes before launching anything
    rc = L.gpgomea_grad_consts(fake, 4, 15, fake, 8, fake, 2, 1000, 1000, fake,
                               gg.FP64_NODES, fake, None, fake, None, fake, ws_need, None)
    assert rc == _lib.E_UNSUPPORTED


def test_single_hip_runtime_in_process():
    """The library shares torch's HIP runtime (one runtime, one device view)."""
    import torch  # noqa: F401
    rts = _lib.hip_runtimes()
    assert len(rts) == 1, rts


def test_tuning_file_roundtrip(tmp_path):
    """A tuning file is read line by line; malformed entries are skipped and an
    unreadable path is an argument error."""
    import paper_2605_30954_amd as gg
    f = tmp_path / "tune.json"
    f.write_text('{"gpgomea_tuning": 1, "entries": [\n'
                 '  {"table": "fwd", "fp64": 0, "Lcls": 5, "F": 10, "Ncls": 16, "Mcls": 10, "grad": 0, '
                 '"K": 8, "R": 1024, "G": 16},\n'
                 '  {"table": "adj", "fp64": 0, "Lcls": 5, "F": 10, "Ncls": 16, "Mcls": 10, "grad": 1, '
                 '"K": 4, "R": 512, "G": 16},\n'
                 '  {"table": "adj", "fp64": 0, "Lcls": 5, "F": 10},\n'
                 '  {"table": "fwd", "fp64": 0, "Lcls": 5, "F": 10, "Ncls": 16, "Mcls": 10, "grad": 0, '
                 '"K": 0, "R": 1024, "G": 16}\n]}\n')
    assert gg.load_tuning(f) == 2
    with pytest.raises(gg.LibraryError):
        gg.load_tuning(tmp_path / "missing.json")
