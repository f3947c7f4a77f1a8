"""The batched GOM loop (Alg. 1) and its FOS, on the CPU: the evaluation is
the oracle, passed in through the loop's ``evaluate`` hook, so what is tested
here is the host logic (variation, change detection, accept/revert)."""
import math

import numpy as np
import pytest

from oracle import codec, fitness as OF, tree as OT
from paper_2605_30954_amd.gom import GOM, proximity_fos
from synth import get_config, make_dataset, sample_population


def test_fos_of_a_height_2_template_by_hand():
    # slots 0..6, children of i at 2i+1, 2i+2.  UPGMA on tree distance:
    # {0,1} (d 1, first pair), {2,5} (d 1), {0,1}+3 (avg 1.5, first in row
    # order), {2,5}+6 (avg 1.5), {0,1,3}+4 (avg 5/3); the root is dropped
    want = [(i,) for i in range(7)] + [(0, 1), (2, 5), (0, 1, 3), (2, 5, 6), (0, 1, 3, 4)]
    assert list(proximity_fos(2)) == want


@pytest.mark.parametrize("h", [3, 6])
def test_fos_is_a_linkage_tree_without_its_root(h):
    T = 2 ** (h + 1) - 1
    fos = [set(s) for s in proximity_fos(h)]
    assert len(fos) == 2 * T - 2
    assert all(len(s) < T for s in fos)
    for a in range(len(fos)):                     # laminar: disjoint or nested
        for b in range(a):
            x, y = fos[a], fos[b]
            assert not (x & y) or x <= y or y <= x
    for k in range(T, len(fos)):                  # each cluster = union of two earlier ones
        kids = [s for s in fos[:k] if s < fos[k] and not any(s < t < fos[k] for t in fos[:k])]
        assert len(kids) == 2 and kids[0] | kids[1] == fos[k]


def _oracle_fitness(genes, gc, h, X, y):
    r = OF.evaluate_population(genes, gc, h, X, y)
    return np.where(r["status"] == 0, r["fitness"], math.inf)


def test_gom_generation_against_the_oracle():
    cfg = get_config(1)
    X, y = make_dataset(cfg, N=300)
    genes, gc, _ = sample_population(cfg, M=24)
    h = cfg.heights[0]
    steps = []

    def evaluate(batch):
        return _oracle_fitness(batch["genes"], batch["gene_consts"], batch["height"], X, y)

    def on_step(st):
        (Vg, Vc), (Bg, Bc) = st["varied"], st["backup"]
        for j in st["touched"]:
            differs = codec.encode_one(Vg[j], Vc[j], h) != codec.encode_one(Bg[j], Bc[j], h)
            assert differs == (j in st["changed"]), (st["fos_index"], j)
        if st["changed"].size:
            np.testing.assert_array_equal(
                st["f_old"], _oracle_fitness(Bg[st["changed"]], Bc[st["changed"]], h, X, y))
            assert np.array_equal(st["accepted"], st["f_new"] <= st["f_old"])
        steps.append(st["changed"].size)

    gom = GOM(genes, gc, h, X=None, y=None, seed=3, evaluate=evaluate, on_step=on_step)
    f0 = gom.fitness.copy()
    for _ in range(2):
        stats = gom.generation()
        assert stats["evaluated"] == sum(stats["batch_sizes"])
        assert stats["accepted"] <= stats["evaluated"]
    assert sum(steps) == gom.evaluations - 24 and len(steps) > 0
    # the tracked fitness is the final population's, and nobody got worse
    np.testing.assert_array_equal(gom.fitness, _oracle_fitness(gom.genes, gom.gc, h, X, y))
    assert np.all(gom.fitness <= f0)
    assert gom.fitness.min() < f0.min() or np.all(gom.fitness == f0)
    # the kept programs are the final genotypes' encodings
    for j in range(24):
        syms, consts = codec.encode_one(gom.genes[j], gom.gc[j], h)
        assert gom.ops[j, : len(syms)].tolist() == syms
        assert np.all(gom.ops[j, len(syms):] == -1)
