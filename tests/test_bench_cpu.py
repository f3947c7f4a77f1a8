"""The benchmark's host-side bookkeeping, checked without a GPU: the
algorithmic lane-op count that is the roofline's numerator (against counts
done by hand from its stated rule) and the HBM-traffic summary built from
rocprofv3 counter files (scaling by the copy probe, the record's validity
keys)."""
import csv
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from oracle import opset as O  # noqa: E402

C, X0, X1 = O.CONST, O.VAR0, O.VAR0 + 1


def _ops(*progs, L=8):
    a = np.full((len(progs), L), -1, np.int8)
    for i, p in enumerate(progs):
        a[i, : len(p)] = p
    return a


def test_program_work_counts_by_hand():
    c = bench.OP_COST
    mom = c["moments"]
    progs = _ops([X0, X1, O.ADD],            # no constant: no gradient work
                 [C, X0, O.MUL],             # c * x0: the product, one chain product
                 [C, X0, O.DIV, O.SIN],      # sin(c / x0)
                 [C, X0, O.ADD],             # c + x0: the partial of + is 1, no product
                 [C, X0, O.MUL],             # bad program (status 2): nothing
                 [C, X0, O.MUL])             # b = 0: forward only
    status = np.array([0, 0, 0, 0, 2, 0])
    s1 = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 0.0])
    nconst = np.array([0, 1, 1, 1, 1, 1])
    fwd, adj = bench.program_work(progs, status, s1, nconst, c)
    want_fwd = ((c["add"] + mom) + (c["mul"] + mom) + (c["div"] + c["sin"] + mom)
                + (c["add"] + mom) + (c["mul"] + mom))
    # sin(c/x0): the division and its partials (a division and a product),
    # one chain product below the sine; the sine, its partial (a cosine) and
    # one chain product
    want_adj = ((c["mul"] + c["mul"])
                + (c["div"] + c["div"] + c["mul"] + c["mul"] + c["sin"] + c["cos"] + c["mul"])
                + c["add"])
    assert fwd == pytest.approx(want_fwd, rel=1e-12)
    assert adj == pytest.approx(want_adj, rel=1e-12)


def test_program_work_counts_constants_on_both_sides():
    c = bench.OP_COST
    # (c0 * x0) * (c1 + x1): the outer product has constants on both sides, so
    # two chain products; the inner + adds none
    progs = _ops([C, X0, O.MUL, C, X1, O.ADD, O.MUL])
    fwd, adj = bench.program_work(progs, np.array([0]), np.array([1.0]), np.array([2]), c)
    assert fwd == pytest.approx(2 * c["mul"] + c["add"] + c["moments"])
    assert adj == pytest.approx((c["mul"] + c["mul"]) + c["add"] + (c["mul"] + 2 * c["mul"]))


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_pmc_summary_scales_by_the_copy_probe(tmp_path, monkeypatch):
    mb = 256
    copy = mb << 20
    adj = "void gg::k_adj_path<4, 4, 4, 16, true, float, false>(gg::AdjParams)"
    part = "gg::k_adj_partition(gg::ProgMeta const*)"
    f_csv, w_csv = str(tmp_path / "f.csv"), str(tmp_path / "w.csv")
    # FETCH_SIZE counts half the probe's bytes, WRITE_SIZE all of them; a
    # small copy (below a quarter of the probe) is not taken for the probe
    _write_counters(f_csv, "FETCH_SIZE", [("__amd_rocclr_copyBuffer", copy / 2 / 1024),
                                          ("__amd_rocclr_copyBuffer", 4.0),
                                          (adj, 1000.0), (adj, 3000.0), (adj, 2000.0), (part, 10.0),
                                          ("gg::k_fused_fwd", 9e9)])
    _write_counters(w_csv, "WRITE_SIZE", [("__amd_rocclr_copyBuffer", copy / 1024), (adj, 50.0), (part, 1.0)])
    tuning = str(tmp_path / "tune.json")
    with open(tuning, "w") as fh:
        fh.write('{"entries": []}\n')
    out_json = str(tmp_path / "traffic.json")
    monkeypatch.setattr(bench, "traffic_file", lambda w: out_json)
    t = bench.pmc_summary(f_csv, w_csv, copy, out_json, 5, tuning)
    assert t["FETCH_SIZE"]["scale"] == pytest.approx(2.0)
    assert t["WRITE_SIZE"]["scale"] == pytest.approx(1.0)
    # medians per kernel (2000 KiB and 10 KiB fetched; 50 and 1 written)
    assert t["FETCH_SIZE"]["adjoint_bytes"] == pytest.approx(2.0 * 2010 * 1024)
    assert t["WRITE_SIZE"]["adjoint_bytes"] == pytest.approx(51 * 1024)
    assert bench.load_traffic(5, tuning) == pytest.approx(t["adjoint_traffic_bytes"])
    assert bench.load_traffic(4, tuning) is None            # another workload
    with open(tuning, "a") as fh:
        fh.write(" ")
    assert bench.load_traffic(5, tuning) is None            # another tuning file

