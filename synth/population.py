"""Seeded template genotypes.

A genotype is a fixed-length, heap-ordered string of symbols laid on a full
binary template of height h (2^(h+1)-1 slots; children of slot i at 2i+1 and
2i+2; leaves at depth h).  The paper's individuals have exactly this form
(Section 3.1); it does not describe initialisation, so half of each population
is sampled "full" (every non-leaf slot an operator) and half "grow" (a non-leaf
slot is a terminal with probability |T|/(|T|+|F|), |T| = number of variables + 1
for the constant).  A terminal is a constant with probability 1/2, otherwise a
uniformly drawn variable.  Leaf slots hold terminals only, and the root is
always an operator.  Unused (intron) slots keep whatever was drawn.

Genotypes of mixed heights share one array of stride 2^(H+1)-1 (H = the largest
height); slots past an individual's own template are PAD.
"""
import numpy as np

from . import symbols as S
from .configs import Config
from .data import rng_for, STREAM_POP, STREAM_GOM


def template_size(h: int) -> int:
    return 2 ** (h + 1) - 1


def _depths(T: int) -> np.ndarray:
    return np.floor(np.log2(np.arange(T) + 1)).astype(np.int64)


def _sample_fixed_height(rng, M, h, funcs, F, erc_lo, erc_hi):
    T = template_size(h)
    depth = _depths(T)
    is_leaf = depth == h
    full = rng.random(M) < 0.5
    u = rng.random((M, T))
    p_term = (F + 1) / (F + 1 + len(funcs))
    is_func = (~is_leaf)[None, :] & (full[:, None] | (u >= p_term))
    is_func[:, 0] = True
    fchoice = np.asarray(funcs, dtype=np.int64)[rng.integers(0, len(funcs), (M, T))]
    is_const = rng.random((M, T)) < 0.5
    vchoice = S.VAR0 + rng.integers(0, F, (M, T))
    cvals = rng.uniform(erc_lo, erc_hi, (M, T)).astype(np.float32)
    genes = np.where(is_func, fchoice, np.where(is_const, S.CONST, vchoice)).astype(np.int8)
    gconst = np.where(genes == S.CONST, cvals, np.float32(0)).astype(np.float32)
    return genes, gconst


def sample_population(cfg: Config, M: int = None, salt: int = 0, heights=None):
    """Return (genes int8 [M, T], gene_consts f32 [M, T], heights int8 [M]).

    T = 2^(H+1)-1 for the largest height H of the workload.  ``heights``
    overrides the per-individual heights.
    """
    M = cfg.M if M is None else int(M)
    rng = rng_for(cfg.cid, STREAM_POP, salt)
    if heights is None:
        if len(cfg.heights) == 1:
            heights = np.full(M, cfg.heights[0], dtype=np.int8)
        else:
            heights = np.asarray(cfg.heights, dtype=np.int8)[rng.integers(0, len(cfg.heights), M)]
    heights = np.asarray(heights, dtype=np.int8)
    H = int(heights.max())
    T = template_size(H)
    genes = np.full((M, T), S.PAD, dtype=np.int8)
    gconst = np.zeros((M, T), dtype=np.float32)
    for h in sorted(set(heights.tolist())):
        idx = np.nonzero(heights == h)[0]
        g, c = _sample_fixed_height(rng, len(idx), int(h), cfg.funcs, cfg.F, cfg.erc_lo, cfg.erc_hi)
        genes[idx, : template_size(h)] = g
        gconst[idx, : template_size(h)] = c
    if cfg.variant_frac > 0:
        genes, gconst, heights = gom_variants(cfg, genes, gconst, heights, cfg.variant_frac, salt)
    return genes, gconst, heights


def _fos_subset(r: int, h: int):
    """Subset number r of a node-proximity style family: parent+children
    triplets for the 2^h - 1 internal slots, then the 2^h single leaves."""
    n_int = 2 ** h - 1
    if r < n_int:
        return np.array([r, 2 * r + 1, 2 * r + 2])
    return np.array([r])


def _active(genes_row, gconst_row, slot=0):
    """The active tree under ``slot`` as a postfix tuple of (symbol, constant
    bits): what an encoder keeps of the genotype (structure only; a unary
    operator's operand is its left child)."""
    g = int(genes_row[slot])
    if 0 <= g < S.CONST:
        kids = (2 * slot + 1,) if g in S.UNARY else (2 * slot + 1, 2 * slot + 2)
        out = ()
        for k in kids:
            out += _active(genes_row, gconst_row, k)
        return out + ((g, 0),)
    bits = int(np.float32(gconst_row[slot]).view(np.int32)) if g == S.CONST else 0
    return ((g, bits),)


def gom_variants(cfg: Config, genes, gconst, heights, frac: float, salt: int = 0):
    """Replace a fraction of the batch by GOM-style offspring.

    An offspring clones a random parent of the same height and copies ONE
    subset of template slots from a random donor of that height (the variation
    step of Alg. 1), redrawn until the copy changes the active tree (Section
    3.1: only a change to an active part is evaluated), so every offspring is
    a new program.  The batch order is shuffled at the end.
    """
    rng = rng_for(cfg.cid, STREAM_GOM, salt)
    M = genes.shape[0]
    n_var = int(round(frac * M))
    n_fresh = M - n_var
    genes = genes.copy()
    gconst = gconst.copy()
    heights = heights.copy()
    fresh_by_h = {}
    for i in range(n_fresh):
        fresh_by_h.setdefault(int(heights[i]), []).append(i)
    for v in range(n_fresh, M):
        for _ in range(1000):
            p = int(rng.integers(0, n_fresh))
            h = int(heights[p])
            pool = fresh_by_h[h]
            d = pool[int(rng.integers(0, len(pool)))]
            sub = _fos_subset(int(rng.integers(0, template_size(h))), h)
            child_g, child_c = genes[p].copy(), gconst[p].copy()
            child_g[sub] = genes[d, sub]
            child_c[sub] = gconst[d, sub]
            if _active(child_g, child_c) != _active(genes[p], gconst[p]):
                break
        genes[v], gconst[v] = child_g, child_c
        heights[v] = h
    perm = rng.permutation(M)
    return genes[perm], gconst[perm], heights[perm]
