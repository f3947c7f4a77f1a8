"""Pins of the oracle's encoder / decoder (Section 3.2, Fig. 1)."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import codec, opset as O, tree as TR

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig1_example.json")


def fig1():
    with open(GOLD) as f:
        g = json.load(f)
    genes = np.array(g["genes"], dtype=np.int8)
    gc = np.array(g["gene_consts"], dtype=np.float32)
    return g, genes, gc


def test_fig1_encoding_matches_paper_arrays():
    g, genes, gc = fig1()
    ops, cs, lens, ncs = codec.encode(genes[None], gc[None], g["height"], 15, 8)
    L = int(lens[0])
    assert ops[0, :L].tolist() == g["expected_ops"]
    assert cs[0, : int(ncs[0])].tolist() == g["expected_consts"]
    assert (ops[0, L:] == -1).all() and (cs[0, int(ncs[0]):] == 0).all()
    # map our byte symbols onto the paper's (type, value) rows independently
    types, values, j = [], [], 0
    opnum = g["paper_operator_codes"]
    names = {0: "+", 1: "-", 2: "*", 3: "/", 4: "sin"}
    for t in ops[0, :L]:
        t = int(t)
        if t == 32:
            types.append(1)
            values.append(float(cs[0, j]))
            j += 1
        elif t >= 64:
            types.append(0)
            values.append(t - 64)
        else:
            types.append(2)
            values.append(opnum[names[t]])
    assert types == g["paper_type_row"]
    assert values == g["paper_value_row"]


def test_fig1_active_set_and_intron_operator():
    g, genes, gc = fig1()
    # the figure's active nodes: /, -2, +, x, x1, 4, x0  (slots 0,1,2,5,6,11,12)
    assert TR.active_slots(genes, 3) == [0, 1, 2, 5, 6, 11, 12]
    # an operator may sit at a leaf slot only as an intron (slot 7 holds 'x')
    bad = genes.copy()
    bad[1] = O.SUB  # makes slots 3,4 active; slot 4 (sin) activates leaf slot 9 (x2) -- fine
    bad[3] = O.MUL  # slot 3 is now an active operator with leaf children 7 ('x'), 8
    with pytest.raises(ValueError):
        codec.encode(bad[None], gc[None], 3, 15, 8)


def test_fig1_infix_and_decode():
    g, genes, gc = fig1()
    ops, cs, *_ = codec.encode(genes[None], gc[None], 3, 15, 8)
    assert codec.infix(ops[0], cs[0]) == "(-2.0 / ((4.0 * x0) + x1))"
    dg, dc = codec.decode(ops, cs, 3)
    act = TR.active_slots(genes, 3)
    for i in range(15):
        if i in act:
            assert dg[0, i] == genes[i] and dc[0, i] == gc[i]
        else:
            assert dg[0, i] == -1 and dc[0, i] == 0


def _random_programs(rng, M, h):
    """Random genotypes of height h over all operators (test-local sampler)."""
    T = 2 ** (h + 1) - 1
    genes = np.empty((M, T), dtype=np.int8)
    gc = rng.uniform(-2, 2, (M, T)).astype(np.float32)
    depth = np.floor(np.log2(np.arange(T) + 1))
    for m in range(M):
        for i in range(T):
            if depth[i] == h or rng.random() < 0.3:
                genes[m, i] = O.CONST if rng.random() < 0.5 else O.VAR0 + rng.integers(0, 5)
            else:
                genes[m, i] = rng.integers(0, 11)
    return genes, gc


@pytest.mark.parametrize("h", [1, 2, 3, 5])
def test_roundtrips(h):
    rng = np.random.default_rng(h)
    genes, gc = _random_programs(rng, 60, h)
    L, C = 2 ** (h + 1) - 1, 2 ** h
    ops, cs, lens, ncs = codec.encode(genes, gc, h, L, C)
    dg, dc = codec.decode(ops, cs, h)
    ops2, cs2, lens2, ncs2 = codec.encode(dg, dc, h, L, C)
    assert (ops2 == ops).all() and (cs2.view(np.uint32) == cs.view(np.uint32)).all()
    assert (lens2 == lens).all() and (ncs2 == ncs).all()
    for m in range(len(genes)):
        act = TR.active_slots(genes[m], h)
        assert sorted(np.nonzero(dg[m] != -1)[0].tolist()) == act
        assert (dg[m, act] == genes[m, act]).all()


def all_height2_genotypes():
    """Every height-2 genotype over {+,-,*,/} and {x0, x1, c}: 7^3 * 3^4."""
    inner = [O.ADD, O.SUB, O.MUL, O.DIV, O.VAR0, O.VAR0 + 1, O.CONST]
    leaf = [O.VAR0, O.VAR0 + 1, O.CONST]
    rows = [list(a) + list(b) for a in itertools.product(inner, repeat=3)
            for b in itertools.product(leaf, repeat=4)]
    genes = np.array(rows, dtype=np.int8)
    gc = np.tile(np.arange(1, 8, dtype=np.float32) * 0.5, (len(rows), 1))
    return genes, gc


def test_exhaustive_height2_roundtrip_and_lengths():
    genes, gc = all_height2_genotypes()
    assert len(genes) == 7 ** 3 * 3 ** 4 == 27783
    ops, cs, lens, ncs = codec.encode(genes, gc, 2, 7, 4)
    # closed form of the active length: count the active slots directly
    for m in range(0, len(genes), 97):
        assert lens[m] == len(TR.active_slots(genes[m], 2))
    dg, dc = codec.decode(ops, cs, 2)
    ops2, *_ = codec.encode(dg, dc, 2, 7, 4)
    assert (ops2 == ops).all()
    # postfix invariant: stack effect sums to exactly one value, never underflows
    eff = {**{o: 1 - O.arity(o) for o in range(11)}, O.CONST: 1, O.VAR0: 1, O.VAR0 + 1: 1}
    for m in range(0, len(genes), 13):
        depth = 0
        for t in ops[m, : lens[m]]:
            depth += eff[int(t)]
            assert depth >= 1
        assert depth == 1


def test_malformed_programs_rejected():
    bad = [
        [O.ADD, -1],                        # underflow
        [O.VAR0, O.VAR0, -1],               # two values left
        [O.CONST, 17, -1],                  # unknown symbol
        [-1],                               # empty
    ]
    for b in bad:
        with pytest.raises(ValueError):
            codec.parse(np.array(b, dtype=np.int8), np.zeros(4, np.float32))
