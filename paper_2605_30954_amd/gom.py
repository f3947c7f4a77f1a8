"""Batched Gene-pool Optimal Mixing: the host loop of Alg. 1 that produces the
batches the library evaluates.

One generation, in Alg. 1's order.  The offspring start as clones of the
population (O = P, backup B = P) and each draws its own random order of the
family of subsets (FOS).  The outer loop runs over FOS positions i, the inner
loop over offspring j: offspring j copies the genes (symbols and constant
values) of subset FOS[order_j[i]] from a donor drawn uniformly from P.  An
offspring joins the batch when its active tree changed, i.e. its postfix
program (symbols and constants, introns skipped: Section 3.1's rule that only
a change to an active part is evaluated) differs from its backup's.  The whole
batch goes to the device in one evaluation call; each evaluated offspring
keeps its change when its fitness is not worse than its backup's (f_new <=
f_old), otherwise it reverts to the backup.  A change that touched introns
only is kept without evaluation (the fitness cannot differ).  After the last
FOS position the offspring replace the population.  Forced improvements,
restarts and linkage learning are not part of this loop.

The FOS is a linkage tree over template slots built from node proximity
(Section 3.1): slots are clustered bottom-up by average distance in the template
tree (UPGMA), every cluster formed on the way is a subset, the root (all
slots) is not.
"""
import time
from functools import lru_cache

import numpy as np

from . import encode, eval_batch

__all__ = ["proximity_fos", "GOM"]


def _tree_distance(T):
    """[T, T] number of edges between heap slots a and b of a full binary
    template (children of slot i at 2i+1 and 2i+2)."""
    a = np.repeat(np.arange(T), T).reshape(T, T)
    b = a.T.copy()
    a = a.copy()
    dist = np.zeros((T, T), dtype=np.int64)
    while True:
        diff = a != b
        if not diff.any():
            return dist
        up_a = diff & (a > b)      # the larger index is never shallower: lift it
        up_b = diff & (b > a)
        a[up_a] = (a[up_a] - 1) // 2
        b[up_b] = (b[up_b] - 1) // 2
        dist += up_a | up_b


@lru_cache(maxsize=8)
def proximity_fos(height):
    """The FOS of a height-``height`` template as a tuple of sorted slot
    tuples: the T singletons first, then the T - 2 merged clusters in merge
    order (UPGMA on the template's tree distance; ties go to the lowest
    (row, column) pair)."""
    T = 2 ** (height + 1) - 1
    D = _tree_distance(T).astype(np.float64)
    np.fill_diagonal(D, np.inf)
    size = np.ones(T)
    members = {i: [i] for i in range(T)}
    fos = [(i,) for i in range(T)]
    for _ in range(T - 1):
        k = int(np.argmin(D))
        i, j = divmod(k, T)
        if i > j:
            i, j = j, i
        si, sj = size[i], size[j]
        row = (si * D[i] + sj * D[j]) / (si + sj)
        D[i, :] = row
        D[:, i] = row
        D[i, i] = np.inf
        D[j, :] = np.inf
        D[:, j] = np.inf
        size[i] = si + sj
        members[i] = members[i] + members.pop(j)
        if len(members[i]) < T:
            fos.append(tuple(sorted(members[i])))
    return tuple(fos)


def _fos_masks(fos, T):
    m = np.zeros((len(fos), T), dtype=bool)
    for f, sub in enumerate(fos):
        m[f, list(sub)] = True
    return m


class GOM:
    """Alg. 1 over a population of one template height.

    genes int8 [M, T], gene_consts float32 [M, T]: heap-ordered genotypes of
    height ``height`` (T = 2^(height+1) - 1).  X float32 [F, N] and y float32
    [N] are device tensors that stay resident.  ``evaluate`` replaces the
    library call (for tests of the loop itself): it gets a dict with the
    batch's postfix programs (ops, consts) and genotypes (genes, gene_consts,
    height) and returns float64 fitness [batch].  ``on_step`` (for tests) is
    called after every FOS position that touched an offspring, with the
    touched and evaluated rows, the old and new fitness, the acceptance, and
    copies of the offspring after variation and of the backup before the
    decisions.
    """

    def __init__(self, genes, gene_consts, height, X, y, linear_scaling=True, seed=0,
                 evaluate=None, on_step=None):
        self.height = int(height)
        self.T = 2 ** (self.height + 1) - 1
        genes = np.ascontiguousarray(genes, dtype=np.int8)
        gc = np.ascontiguousarray(gene_consts, dtype=np.float32)
        if genes.shape != gc.shape or genes.shape[1] != self.T:
            raise ValueError(f"genotypes must be [M, {self.T}] for height {self.height}")
        self.M = genes.shape[0]
        self.L_max, self.C_max = self.T, 2 ** self.height
        self.X, self.y = X, y
        self.linear_scaling = linear_scaling
        self.rng = np.random.default_rng(seed)
        self.fos = proximity_fos(self.height)
        self.masks = _fos_masks(self.fos, self.T)
        self.evaluate = evaluate if evaluate is not None else self._device_evaluate
        self.on_step = on_step
        self.genes, self.gc = genes.copy(), gc.copy()
        self.ops, self.cs = self._encode(self.genes, self.gc)
        self.fitness = self._evaluate(self.ops, self.cs, self.genes, self.gc)
        self.evaluations = self.M
        self.history = []

    # -- helpers -----------------------------------------------------------
    def _encode(self, genes, gc):
        ops, cs, _, _ = encode(genes, gc, self.height, self.L_max, self.C_max)
        return ops, cs

    def _device_evaluate(self, batch):
        import torch
        dev = self.X.device
        ops = torch.from_numpy(batch["ops"]).to(dev)
        cs = torch.from_numpy(batch["consts"]).to(dev)
        return eval_batch(ops, cs, self.X, self.y, linear_scaling=self.linear_scaling).cpu().numpy()

    def _evaluate(self, ops, cs, genes, gc):
        if ops.shape[0] == 0:
            return np.zeros(0)
        batch = dict(ops=np.ascontiguousarray(ops), consts=np.ascontiguousarray(cs),
                     genes=genes, gene_consts=gc, height=self.height)
        return np.asarray(self.evaluate(batch), dtype=np.float64)

    # -- one generation ----------------------------------------------------
    def generation(self):
        """Run Alg. 1 once; returns a dict of counts and timings."""
        t_all = time.perf_counter()
        M, T = self.M, self.T
        Pg, Pc = self.genes, self.gc                      # donors come from P
        Og, Oc = Pg.copy(), Pc.copy()                     # offspring
        Bg, Bc = Pg.copy(), Pc.copy()                     # backup
        Bops, Bcs, Bfit = self.ops.copy(), self.cs.copy(), self.fitness.copy()
        order = np.argsort(self.rng.random((M, len(self.fos))), axis=1)
        rows = np.arange(M)
        stats = dict(fos_steps=len(self.fos), evaluated=0, accepted=0, intron_only=0,
                     batch_sizes=[], t_eval=0.0)
        for i in range(len(self.fos)):
            donors = self.rng.integers(0, M, M)
            mask = self.masks[order[:, i]]                               # [M, T]
            Dg, Dc = Pg[donors], Pc[donors]
            touched = np.any(mask & ((Dg != Og) | (Dc.view(np.int32) != Oc.view(np.int32))), axis=1)
            t_idx = rows[touched]
            if t_idx.size == 0:
                stats["batch_sizes"].append(0)
                continue
            Og[t_idx] = np.where(mask[t_idx], Dg[t_idx], Og[t_idx])
            Oc[t_idx] = np.where(mask[t_idx], Dc[t_idx], Oc[t_idx])
            snap = ((Og.copy(), Oc.copy()), (Bg.copy(), Bc.copy())) if self.on_step else None
            ops_t, cs_t = self._encode(Og[t_idx], Oc[t_idx])
            diff = np.any(ops_t != Bops[t_idx], axis=1) | \
                np.any(cs_t.view(np.int32) != Bcs[t_idx].view(np.int32), axis=1)
            ch = t_idx[diff]
            still = t_idx[~diff]                   # intron-only: keep, nothing to evaluate
            Bg[still], Bc[still] = Og[still], Oc[still]
            stats["intron_only"] += int(still.size)
            stats["batch_sizes"].append(int(ch.size))
            if ch.size == 0:
                if self.on_step is not None:
                    self.on_step(dict(fos_index=i, touched=t_idx, changed=ch, f_new=np.zeros(0),
                                      f_old=np.zeros(0), accepted=np.zeros(0, bool), varied=snap[0],
                                      backup=snap[1]))
                continue
            ops_c, cs_c = ops_t[diff], cs_t[diff]
            t0 = time.perf_counter()
            f_new = self._evaluate(ops_c, cs_c, Og[ch], Oc[ch])
            stats["t_eval"] += time.perf_counter() - t0
            f_old = Bfit[ch].copy()
            acc = f_new <= f_old
            a_idx, r_idx = ch[acc], ch[~acc]
            Bg[a_idx], Bc[a_idx] = Og[a_idx], Oc[a_idx]
            Bops[a_idx], Bcs[a_idx] = ops_c[acc], cs_c[acc]
            Bfit[a_idx] = f_new[acc]
            Og[r_idx], Oc[r_idx] = Bg[r_idx], Bc[r_idx]
            stats["evaluated"] += int(ch.size)
            stats["accepted"] += int(a_idx.size)
            if self.on_step is not None:
                self.on_step(dict(fos_index=i, touched=t_idx, changed=ch, f_new=f_new, f_old=f_old,
                                  accepted=acc, varied=snap[0], backup=snap[1]))
        # every offspring now equals its backup (accepted, reverted or intron-only)
        self.genes, self.gc = Og, Oc
        self.ops, self.cs, self.fitness = Bops, Bcs, Bfit
        self.evaluations += stats["evaluated"]
        stats["t_total"] = time.perf_counter() - t_all
        self.history.append(stats)
        return stats
