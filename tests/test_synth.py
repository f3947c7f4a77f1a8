"""The input generators' structural helpers, checked against the oracle's
encoder: the active-tree walk that the GOM-style variants use to make sure
every offspring differs from its parent in an active part (Section 3.1)."""
import numpy as np

from oracle import codec
from synth import get_config, sample_population
from synth.population import _active


def test_active_walk_matches_the_oracle_encoder():
    for cid in (1, 3, 5):
        cfg = get_config(cid)
        genes, gc, hs = sample_population(cfg, M=200, salt=9)
        for m in range(genes.shape[0]):
            syms, consts = codec.encode_one(genes[m], gc[m], int(hs[m]))
            act = _active(genes[m], gc[m])
            assert [s for s, _ in act] == syms
            bits = [b for s, b in act if s == 32]
            assert bits == [int(np.float32(c).view(np.int32)) for c in consts]


def test_gom_offspring_batch_has_fresh_and_varied_programs():
    cfg = get_config(3)
    genes, gc, hs = sample_population(cfg, M=400, salt=2)
    progs = {_active(genes[m], gc[m]) for m in range(400)}
    # 30 % offspring, each a different active tree from its parent: almost
    # every program of the batch is distinct
    assert len(progs) >= 0.95 * 400
