"""Seeded synthetic workloads for evolving graphs.

This module only draws random graphs, random update streams and random
Gaussian sketch matrices.  It holds none of the eigen-update arithmetic, so the
GPU path, the tests and the benchmark can all share it.

Graph model (paper Sec. 2, eq. adj_update): at every step a graph with ``n``
nodes receives a set of undirected edge changes and ``S`` appended nodes with
ids ``n .. n+S-1``.  A change is a pair ``(i, j)`` with ``i < j`` and a sign
``+1`` (insert a missing edge) or ``-1`` (delete an existing edge); an edge that
touches an appended node is always an insertion.

Workload families (all sizes are parameters; the presets below give the shapes
the method is measured on):

* ``sbm_small``: dense Bernoulli stochastic block model with equal blocks,
  grown by new nodes wired with the same block probabilities, plus uniform
  insertions among non-adjacent old pairs and uniform deletions of old edges.
* ``sbm_large``: O(m) stochastic block model with Dirichlet block proportions
  (binomial edge count per block pair, uniform endpoints), grown by new nodes
  with Poisson(4) edges each (80 % inside their own block) plus uniform
  old-old insertions at the same intra/inter ratio.
* ``chung_lu``: power-law expected degrees (Pareto weights with pdf exponent
  gamma, capped), edges drawn with endpoints proportional to the weights,
  duplicates and self-loops dropped, nodes outside the largest component
  attached by one edge.  Updates either insert/delete a fraction of the edges
  or append nodes whose partners are drawn proportional to the weights.

* ``sbm_expansion``: a Bernoulli SBM on all N nodes (uniform random clusters),
  revealed by expansion only: the subgraph induced by n0 random nodes, then
  batches of further random nodes with all their edges; returns the clusters
  too, for the spectral-clustering check.
Node ids are randomly permuted at t=0 so that neighbouring ids carry no block
locality; appended nodes take the next ids.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

BASE_ENTROPY = 260319439

# stream ids inside a SeedSequence
_GRAPH, _DELTA, _OMEGA, _ARRIVAL = 0, 1, 2, 3


def rng_for(cfg_id: int, graph_id: int, step: int, stream: int) -> np.random.Generator:
    """A numpy Generator seeded from (cfg, graph, step, stream)."""
    ss = np.random.SeedSequence([BASE_ENTROPY, int(cfg_id), int(graph_id), int(step), int(stream)])
    return np.random.default_rng(ss)


# --------------------------------------------------------------------------------------
# edge-set helpers (canonical undirected keys i < j encoded as i * KEY_BASE + j)
# --------------------------------------------------------------------------------------
KEY_BASE = np.int64(1) << np.int64(32)


def _keys(i: np.ndarray, j: np.ndarray) -> np.ndarray:
    lo = np.minimum(i, j).astype(np.int64)
    hi = np.maximum(i, j).astype(np.int64)
    return lo * KEY_BASE + hi


def _unkey(k: np.ndarray):
    return (k // KEY_BASE).astype(np.int64), (k % KEY_BASE).astype(np.int64)


def csr_from_keys(n: int, keys: np.ndarray):
    """Symmetric CSR (both triangles, sorted columns) from canonical edge keys."""
    i, j = _unkey(keys)
    rows = np.concatenate([i, j])
    cols = np.concatenate([j, i])
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order].astype(np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    np.cumsum(rowptr, out=rowptr)
    return rowptr, cols


@dataclasses.dataclass
class Delta:
    """One update: ``n_new`` appended nodes and undirected changes (i < j, sign)."""
    n_old: int
    n_new: int
    i: np.ndarray  # int64
    j: np.ndarray  # int64
    sign: np.ndarray  # int8, +1 insert / -1 delete

    @property
    def n_changes(self) -> int:
        return int(self.i.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    cfg_id: int
    n0: int
    rowptr0: np.ndarray
    col0: np.ndarray
    deltas: List[Delta]
    keys_final: Optional[np.ndarray] = None

    def keys_at(self, t: int) -> np.ndarray:
        """Canonical edge keys of the graph after ``t`` updates."""
        keys = _keys_from_csr(self.rowptr0, self.col0)
        for d in self.deltas[:t]:
            keys = apply_delta_keys(keys, d)
        return keys

    def n_at(self, t: int) -> int:
        n = self.n0
        for d in self.deltas[:t]:
            n += d.n_new
        return n


def _keys_from_csr(rowptr, col):
    n = rowptr.shape[0] - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    c = col.astype(np.int64)
    m = rows < c
    return np.sort(rows[m] * KEY_BASE + c[m])


def apply_delta_keys(keys: np.ndarray, d: Delta) -> np.ndarray:
    k = _keys(d.i, d.j)
    ins = k[d.sign > 0]
    dele = k[d.sign < 0]
    out = keys
    if dele.size:
        out = out[~np.isin(out, dele, assume_unique=False)]
    if ins.size:
        out = np.union1d(out, ins)
    return out


def _dedupe_pairs(i, j, n_exclude_keys=None):
    m = i != j
    k = np.unique(_keys(i[m], j[m]))
    if n_exclude_keys is not None and n_exclude_keys.size:
        k = k[~np.isin(k, n_exclude_keys)]
    return k


def _sample_nonadjacent(rng, keys, lo, hi, count, forbid=None):
    """``count`` distinct uniform pairs in [lo, hi) that are not edges in ``keys``."""
    got = np.empty(0, dtype=np.int64)
    while got.size < count:
        need = count - got.size
        a = rng.integers(lo, hi, size=2 * need + 16)
        b = rng.integers(lo, hi, size=2 * need + 16)
        k = _dedupe_pairs(a, b)
        k = k[~np.isin(k, keys)]
        if forbid is not None:
            k = k[~np.isin(k, forbid)]
        k = np.setdiff1d(k, got)
        rng.shuffle(k)
        got = np.concatenate([got, k[:need]])
    return got[:count]


def _delta_from_keys(n_old, n_new, ins_keys, del_keys) -> Delta:
    ins_keys = np.unique(ins_keys)
    del_keys = np.unique(del_keys)
    ii, jj = _unkey(ins_keys)
    di, dj = _unkey(del_keys)
    return Delta(
        n_old=n_old,
        n_new=n_new,
        i=np.concatenate([ii, di]).astype(np.int64),
        j=np.concatenate([jj, dj]).astype(np.int64),
        sign=np.concatenate([np.ones(ii.size, np.int8), -np.ones(di.size, np.int8)]),
    )


# --------------------------------------------------------------------------------------
# small dense SBM (equal blocks, Bernoulli per pair)
# --------------------------------------------------------------------------------------
def sbm_small(n0=2000, blocks=4, p_in=0.05, p_out=0.005, steps=10, new_per_step=100,
              insertions=300, deletions=100, cfg_id=1, graph_id=0) -> Workload:
    rng = rng_for(cfg_id, graph_id, 0, _GRAPH)
    lab = np.repeat(np.arange(blocks), n0 // blocks)
    lab = np.concatenate([lab, rng.integers(0, blocks, n0 - lab.size)])
    iu, ju = np.triu_indices(n0, 1)
    p = np.where(lab[iu] == lab[ju], p_in, p_out)
    m = rng.random(iu.size) < p
    ei, ej = iu[m], ju[m]
    perm = rng.permutation(n0)  # random ids: no block locality in node numbering
    labels = np.empty(n0, dtype=np.int64)
    labels[perm] = lab
    keys = np.unique(_keys(perm[ei], perm[ej]))
    rowptr0, col0 = csr_from_keys(n0, keys)

    deltas = []
    n = n0
    for t in range(1, steps + 1):
        r = rng_for(cfg_id, graph_id, t, _DELTA)
        lab_new = r.integers(0, blocks, new_per_step)
        all_lab = np.concatenate([labels, lab_new])
        ins = []
        # new node wiring: to every node that exists now, and among the new nodes
        for q in range(new_per_step):
            v = n + q
            cand = np.arange(v)
            pp = np.where(all_lab[cand] == lab_new[q], p_in, p_out)
            hit = cand[r.random(cand.size) < pp]
            ins.append(_keys(hit, np.full(hit.size, v)))
        ins_new = np.concatenate(ins) if ins else np.empty(0, np.int64)
        # uniform insertions among non-adjacent old pairs
        ins_old = _sample_nonadjacent(r, keys, 0, n, insertions)
        # uniform deletions of old edges
        dele = r.choice(keys, size=min(deletions, keys.size), replace=False)
        d = _delta_from_keys(n, new_per_step, np.concatenate([ins_new, ins_old]), dele)
        deltas.append(d)
        keys = apply_delta_keys(keys, d)
        labels = all_lab
        n += new_per_step
    return Workload("sbm_small", cfg_id, n0, rowptr0, col0, deltas, keys)


# --------------------------------------------------------------------------------------
# SBM revealed by graph expansion, with its ground-truth clusters
# --------------------------------------------------------------------------------------
def _distinct_pairs(rng, cnt, na, nb, same):
    """cnt distinct pairs drawn uniformly: unordered pairs inside one group of na nodes
    (same) or pairs across groups of na and nb nodes, as flat indices a * (na or nb) + b.
    Uniform draws are merged until cnt distinct ones exist, then cnt of them are kept at
    random: a uniformly random cnt-subset, so that with a binomial cnt every pair is an
    edge independently (a Bernoulli graph)."""
    width = na if same else nb
    got = np.empty(0, np.int64)
    while got.size < cnt:
        m = int((cnt - got.size) * 1.2) + 16
        a = rng.integers(0, na, m)
        b = rng.integers(0, width, m)
        if same:
            keep = a != b
            a, b = np.minimum(a[keep], b[keep]), np.maximum(a[keep], b[keep])
        got = np.unique(np.concatenate([got, a.astype(np.int64) * width + b]))
    if got.size > cnt:
        got = rng.choice(got, cnt, replace=False)
    return got, width


@dataclasses.dataclass
class ClusteredWorkload:
    workload: Workload
    labels: np.ndarray  # cluster of every node of the final graph, by node id


def sbm_expansion(N=10_000, clusters=4, p_in=0.05, p_out=0.005, n0=9_500, steps=10, new_per_step=50,
                  cfg_id=6, graph_id=0) -> ClusteredWorkload:
    """An SBM on N nodes (each node in a uniformly random cluster; a pair is an edge with
    probability p_in inside a cluster and p_out across), revealed by expansion: the graph
    at t = 0 is the subgraph induced by n0 random nodes, and every step adds new_per_step
    further random nodes with all their edges to the nodes present (updates are
    insertions touching new nodes only).  Node ids follow the order of arrival."""
    rng = rng_for(cfg_id, graph_id, 0, _GRAPH)
    lab = rng.integers(0, clusters, N)
    sizes = np.bincount(lab, minlength=clusters).astype(np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    gi, gj = [], []  # edges in the numbering where clusters are contiguous
    for b in range(clusters):
        sb = int(sizes[b])
        if sb >= 2:
            idx, w = _distinct_pairs(rng, rng.binomial(sb * (sb - 1) // 2, p_in), sb, sb, True)
            gi.append(idx // w + offsets[b])
            gj.append(idx % w + offsets[b])
        for c in range(b + 1, clusters):
            sc = int(sizes[c])
            if sb == 0 or sc == 0:
                continue
            idx, w = _distinct_pairs(rng, rng.binomial(sb * sc, p_out), sb, sc, False)
            gi.append(idx // w + offsets[b])
            gj.append(idx % w + offsets[c])
    gi = np.concatenate(gi) if gi else np.empty(0, np.int64)
    gj = np.concatenate(gj) if gj else np.empty(0, np.int64)
    arrival = rng.permutation(N)  # node g of the contiguous numbering gets id arrival[g]
    labels = np.empty(N, dtype=np.int64)
    labels[arrival] = np.repeat(np.arange(clusters), sizes)
    ei, ej = arrival[gi], arrival[gj]
    lo, hi = np.minimum(ei, ej), np.maximum(ei, ej)
    first = hi < n0
    keys = np.unique(_keys(lo[first], hi[first]))
    rowptr0, col0 = csr_from_keys(n0, keys)
    deltas = []
    n = n0
    for _ in range(steps):
        s = min(new_per_step, N - n)
        if s <= 0:
            break
        m = (hi >= n) & (hi < n + s)
        d = _delta_from_keys(n, s, _keys(lo[m], hi[m]), np.empty(0, np.int64))
        deltas.append(d)
        keys = apply_delta_keys(keys, d)
        n += s
    wl = Workload("sbm_expansion", cfg_id, n0, rowptr0, col0, deltas, keys)
    return ClusteredWorkload(wl, labels[:n])


# --------------------------------------------------------------------------------------
# large O(m) SBM with Dirichlet block sizes
# --------------------------------------------------------------------------------------
def _sbm_edges_by_counts(rng, sizes, offsets, p_in, p_out):
    nb = sizes.size
    out_i, out_j = [], []
    for b in range(nb):
        nbb = int(sizes[b])
        if nbb >= 2:
            cnt = rng.binomial(nbb * (nbb - 1) // 2, min(1.0, p_in))
            a = rng.integers(0, nbb, cnt) + offsets[b]
            c = rng.integers(0, nbb, cnt) + offsets[b]
            out_i.append(a)
            out_j.append(c)
        for c2 in range(b + 1, nb):
            cnt = rng.binomial(int(sizes[b]) * int(sizes[c2]), min(1.0, p_out))
            a = rng.integers(0, int(sizes[b]), cnt) + offsets[b]
            c = rng.integers(0, int(sizes[c2]), cnt) + offsets[c2]
            out_i.append(a)
            out_j.append(c)
    return np.concatenate(out_i), np.concatenate(out_j)


def sbm_large(n0=1_000_000, blocks=32, dirichlet=2.0, deg_in=16.0, deg_out=4.0, steps=10,
              new_per_step=10_000, new_deg=4.0, old_insertions=10_000, intra_frac=0.8,
              cfg_id=3, graph_id=0, permute=True) -> Workload:
    """O(m) SBM; ``permute=False`` keeps the initial ids sorted by block (a locality
    reference: the same graph with neighbours close in id space)."""
    rng = rng_for(cfg_id, graph_id, 0, _GRAPH)
    pi = rng.dirichlet(np.full(blocks, dirichlet))
    sizes = rng.multinomial(n0, pi).astype(np.int64)
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    ssq = float(np.sum(sizes.astype(np.float64) ** 2))
    p_in = deg_in * n0 / ssq
    p_out = deg_out * n0 / (float(n0) ** 2 - ssq)
    a, b = _sbm_edges_by_counts(rng, sizes, offsets, p_in, p_out)
    lab_sorted = np.repeat(np.arange(blocks), sizes)
    perm = rng.permutation(n0)
    if not permute:
        perm = np.arange(n0)
    labels = np.empty(n0, dtype=np.int64)
    labels[perm] = lab_sorted
    keys = _dedupe_pairs(perm[a], perm[b])
    del a, b
    rowptr0, col0 = csr_from_keys(n0, keys)

    deltas = []
    n = n0
    for t in range(1, steps + 1):
        r = rng_for(cfg_id, graph_id, t, _DELTA)
        lab_new = r.choice(blocks, size=new_per_step, p=pi)
        all_lab = np.concatenate([labels, lab_new])
        order = np.argsort(all_lab, kind="stable")
        cnt = np.bincount(all_lab, minlength=blocks)
        start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
        # edges incident to new nodes: Poisson(new_deg) each, intra_frac to own block
        k = r.poisson(new_deg, new_per_step)
        src = np.repeat(np.arange(n, n + new_per_step), k)
        own = np.repeat(lab_new, k)
        intra = r.random(src.size) < intra_frac
        tgt = np.empty(src.size, dtype=np.int64)
        # intra: uniform member of own block (old or new)
        pos = (r.random(src.size) * cnt[own]).astype(np.int64)
        tgt[intra] = order[start[own[intra]] + pos[intra]]
        # inter: uniform node of the whole graph outside the own block (redraw clashes)
        ninter = int((~intra).sum())
        own_inter = own[~intra]
        fill = r.integers(0, n + new_per_step, ninter)
        bad = all_lab[fill] == own_inter
        while bad.any():
            fill[bad] = r.integers(0, n + new_per_step, int(bad.sum()))
            bad = all_lab[fill] == own_inter
        tgt[~intra] = fill
        ins_new = _dedupe_pairs(src, tgt)
        # old-old insertions at the same intra/inter ratio
        n_intra = int(round(old_insertions * intra_frac))
        old_order = np.argsort(labels, kind="stable")
        ocnt = np.bincount(labels, minlength=blocks)
        ostart = np.concatenate([[0], np.cumsum(ocnt)[:-1]])
        bsel = r.choice(blocks, size=2 * n_intra + 16, p=ocnt / ocnt.sum())
        u = old_order[ostart[bsel] + (r.random(bsel.size) * ocnt[bsel]).astype(np.int64)]
        v = old_order[ostart[bsel] + (r.random(bsel.size) * ocnt[bsel]).astype(np.int64)]
        ki = _dedupe_pairs(u, v, keys)
        r.shuffle(ki)
        ki = ki[:n_intra]
        u = r.integers(0, n, 4 * (old_insertions - n_intra) + 16)
        v = r.integers(0, n, u.size)
        m = labels[u] != labels[v]
        ko = _dedupe_pairs(u[m], v[m], keys)
        ko = np.setdiff1d(ko, ki)
        r.shuffle(ko)
        ko = ko[: old_insertions - n_intra]
        d = _delta_from_keys(n, new_per_step, np.concatenate([ins_new, ki, ko]), np.empty(0, np.int64))
        deltas.append(d)
        keys = apply_delta_keys(keys, d)
        labels = all_lab
        n += new_per_step
    return Workload("sbm_large", cfg_id, n0, rowptr0, col0, deltas, keys)


# --------------------------------------------------------------------------------------
# Chung-Lu power-law graphs
# --------------------------------------------------------------------------------------
def pareto_weights(rng, n, gamma, mean, cap):
    """Capped Pareto weights with pdf exponent ``gamma`` (tail index gamma-1), scaled so
    that the capped mean equals ``mean``."""
    a = gamma - 1.0
    u = rng.random(n)
    base = (1.0 - u) ** (-1.0 / a)  # Pareto with x_m = 1

    def capped_mean(xm):
        return float(np.minimum(xm * base, cap).mean())

    lo, hi = 1e-6, mean
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if capped_mean(mid) < mean:
            lo = mid
        else:
            hi = mid
    return np.minimum(hi * base, cap), hi


def _chung_lu_keys(rng, w):
    n = w.size
    total = float(w.sum())
    m = rng.poisson(total / 2.0)
    p = w / total
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    a = np.searchsorted(cdf, rng.random(m), side="right")
    b = np.searchsorted(cdf, rng.random(m), side="right")
    return _dedupe_pairs(a.astype(np.int64), b.astype(np.int64))


def _connect(rng, n, keys, w):
    """Attach every node outside the largest component by one edge to an LCC node
    drawn proportional to ``w``."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    i, j = _unkey(keys)
    g = sp.coo_matrix((np.ones(i.size), (i, j)), shape=(n, n))
    ncomp, lab = connected_components(g, directed=False)
    if ncomp == 1:
        return keys
    big = np.argmax(np.bincount(lab))
    lcc = np.flatnonzero(lab == big)
    outside = np.flatnonzero(lab != big)
    pw = w[lcc] / w[lcc].sum()
    tgt = lcc[np.searchsorted(np.cumsum(pw), rng.random(outside.size) * (1 - 1e-12), side="right")]
    return np.union1d(keys, _keys(outside, tgt))


def chung_lu(n0=100_000, gamma=2.5, mean=16.0, cap=2000.0, steps=20, ins_frac=0.005,
             del_frac=0.002, grow_frac=0.0, cfg_id=2, graph_id=0) -> Workload:
    """Chung-Lu graph with edge-churn updates (``grow_frac == 0``) or node-growth
    updates (``grow_frac > 0``: that fraction of n appended per step, each new node
    with max(1, Poisson(w)) partners drawn proportional to the weights)."""
    rng = rng_for(cfg_id, graph_id, 0, _GRAPH)
    if cap is None:
        cap = float(np.sqrt(mean * n0))
    w, xm = pareto_weights(rng, n0, gamma, mean, cap)
    keys = _chung_lu_keys(rng, w)
    keys = _connect(rng, n0, keys, w)
    rowptr0, col0 = csr_from_keys(n0, keys)
    deltas = []
    n = n0
    for t in range(1, steps + 1):
        r = rng_for(cfg_id, graph_id, t, _DELTA)
        if grow_frac > 0:
            s = int(round(grow_frac * n0))
            wn = np.minimum(xm * (1.0 - r.random(s)) ** (-1.0 / (gamma - 1.0)), cap)
            deg = np.maximum(1, r.poisson(wn))
            src = np.repeat(np.arange(n, n + s), deg)
            cdf = np.cumsum(w / w.sum())
            cdf[-1] = 1.0
            tgt = np.searchsorted(cdf, r.random(src.size), side="right").astype(np.int64)
            ins = _dedupe_pairs(src, tgt)
            d = _delta_from_keys(n, s, ins, np.empty(0, np.int64))
            w = np.concatenate([w, wn])
            n += s
        else:
            m_now = keys.size
            n_ins = int(round(ins_frac * m_now))
            n_del = int(round(del_frac * m_now))
            ins = _sample_nonadjacent(r, keys, 0, n, n_ins)
            deg = np.bincount(_unkey(keys)[0], minlength=n) + np.bincount(_unkey(keys)[1], minlength=n)
            cand = r.permutation(keys)
            dele = []
            for kk in cand:
                if len(dele) == n_del:
                    break
                a, b = int(kk // KEY_BASE), int(kk % KEY_BASE)
                if deg[a] > 1 and deg[b] > 1:
                    deg[a] -= 1
                    deg[b] -= 1
                    dele.append(kk)
            d = _delta_from_keys(n, 0, ins, np.asarray(dele, dtype=np.int64))
        deltas.append(d)
        keys = apply_delta_keys(keys, d)
    return Workload("chung_lu", cfg_id, n0, rowptr0, col0, deltas, keys)


# --------------------------------------------------------------------------------------
# many independent graphs with a stream of update requests (serving)
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class ServingGraph:
    graph_id: int
    family: str  # "sbm" or "chunglu"
    k: int
    workload: Workload  # the initial graph and its requests, in order


class _EdgeSet:
    """Membership of canonical keys: a sorted base array plus recent additions, merged
    from time to time (insert-only streams)."""

    def __init__(self, keys):
        self.base = np.sort(keys)
        self.extra = []
        self.count = int(self.base.size)

    def contains(self, k):
        pos = np.searchsorted(self.base, k)
        hit = (pos < self.base.size) & (self.base[np.minimum(pos, self.base.size - 1)] == k)
        for e in self.extra:
            hit |= np.isin(k, e)
        return hit

    def add(self, k):
        self.extra.append(np.asarray(k, dtype=np.int64))
        self.count += int(k.size)
        if len(self.extra) >= 8:
            self.base = np.union1d(self.base, np.concatenate(self.extra))
            self.extra = []


def serving_graph(graph_id: int, requests: int, scale: float = 1.0, cfg_id: int = 4) -> ServingGraph:
    """One graph of the many-graph serving mix and ``requests`` updates for it.

    Family Bernoulli(1/2): SBM (8-32 blocks, Dirichlet(2) proportions, 80 % of the edges
    inside blocks) or Chung-Lu (pdf exponent 2.5).  Mean degree uniform in 8..32,
    n0 ~ LogNormal(ln 5e4, 1) clipped to [1e4, 5e5] (times ``scale``), K uniform in
    {8, 16, 32}.  Each request appends round(U[0.1, 1] % of n) nodes, wired per family
    (SBM: Poisson(d/2) partners, 80 % in the node's own block; Chung-Lu: max(1,
    Poisson(w)) partners proportional to the weights), plus round(U[0.1, 1] % of the
    edge count) uniform insertions among non-adjacent existing pairs."""
    rng = rng_for(cfg_id, graph_id, 0, _GRAPH)
    family = "sbm" if rng.random() < 0.5 else "chunglu"
    n0 = int(np.clip(np.exp(rng.normal(np.log(5e4), 1.0)), 1e4, 5e5) * scale)
    n0 = max(n0, 64)
    d = int(rng.integers(8, 33))
    k = int(rng.choice([8, 16, 32]))
    if family == "sbm":
        blocks = int(rng.integers(8, 33))
        pi = rng.dirichlet(np.full(blocks, 2.0))
        sizes = rng.multinomial(n0, pi).astype(np.int64)
        offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        ssq = float(np.sum(sizes.astype(np.float64) ** 2))
        p_in = 0.8 * d * n0 / ssq
        p_out = 0.2 * d * n0 / max(float(n0) ** 2 - ssq, 1.0)
        a, b = _sbm_edges_by_counts(rng, sizes, offsets, p_in, p_out)
        perm = rng.permutation(n0)
        labels = np.empty(n0, dtype=np.int64)
        labels[perm] = np.repeat(np.arange(blocks), sizes)
        keys = _dedupe_pairs(perm[a], perm[b])
        w = None
    else:
        cap = float(np.sqrt(d * n0))
        w, xm = pareto_weights(rng, n0, 2.5, float(d), cap)
        keys = _connect(rng, n0, _chung_lu_keys(rng, w), w)
        labels = None
    rowptr0, col0 = csr_from_keys(n0, keys)
    es = _EdgeSet(keys)
    deltas = []
    n = n0
    for t in range(1, requests + 1):
        r = rng_for(cfg_id, graph_id, t, _DELTA)
        s = max(1, int(round(r.uniform(0.001, 0.01) * n)))
        n_ins = int(round(r.uniform(0.001, 0.01) * es.count))
        if family == "sbm":
            lab_new = r.choice(pi.size, size=s, p=pi)
            all_lab = np.concatenate([labels, lab_new])
            order = np.argsort(all_lab, kind="stable")
            cnt = np.bincount(all_lab, minlength=pi.size)
            start = np.concatenate([[0], np.cumsum(cnt)[:-1]])
            deg = r.poisson(d / 2.0, s)
            src = np.repeat(np.arange(n, n + s), deg)
            own = np.repeat(lab_new, deg)
            intra = r.random(src.size) < 0.8
            tgt = r.integers(0, n + s, src.size)
            pos = (r.random(src.size) * cnt[own]).astype(np.int64)
            tgt[intra] = order[start[own[intra]] + pos[intra]]
            labels = all_lab
        else:
            wn = np.minimum(xm * (1.0 - r.random(s)) ** (-1.0 / 1.5), cap)
            deg = np.maximum(1, r.poisson(wn))
            src = np.repeat(np.arange(n, n + s), deg)
            cdf = np.cumsum(w / w.sum())
            cdf[-1] = 1.0
            tgt = np.searchsorted(cdf, r.random(src.size), side="right").astype(np.int64)
            w = np.concatenate([w, wn])
        ins_new = _dedupe_pairs(src, tgt)
        u = r.integers(0, n, 2 * n_ins + 16)
        v = r.integers(0, n, u.size)
        ko = _dedupe_pairs(u, v)
        ko = ko[~es.contains(ko)]
        r.shuffle(ko)
        ko = ko[:n_ins]
        dl = _delta_from_keys(n, s, np.concatenate([ins_new, ko]), np.empty(0, np.int64))
        deltas.append(dl)
        es.add(_keys(dl.i, dl.j))
        n += s
    wl = Workload(f"serving_{family}", cfg_id, n0, rowptr0, col0, deltas)
    return ServingGraph(graph_id, family, k, wl)


def arrivals(rate: float, count: int, graphs: int, seed: int, cfg_id: int = 4):
    """Poisson arrival times (seconds from the start) and uniform target graphs."""
    r = rng_for(cfg_id, seed, 0, _ARRIVAL)
    t = np.cumsum(r.exponential(1.0 / rate, count))
    g = r.integers(0, graphs, count)
    return t, g


def omega(cfg_id: int, graph_id: int, step: int, rows: int, cols: int) -> np.ndarray:
    """The Gaussian test matrix of the randomized range finder, i.i.d. N(0,1), FP64,
    ``rows x cols`` row-major.  Passed to both the oracle and the GPU path."""
    return rng_for(cfg_id, graph_id, step, _OMEGA).standard_normal((rows, cols))


def random_orthonormal(n: int, k: int, seed: int = 0) -> np.ndarray:
    """A random n x k matrix with orthonormal columns (Gaussian then QR)."""
    g = np.random.default_rng(np.random.SeedSequence([BASE_ENTROPY, 99, seed])).standard_normal((n, k))
    q, _ = np.linalg.qr(g)
    return np.ascontiguousarray(q)


# --------------------------------------------------------------------------------------
# presets matching the measured configurations
# --------------------------------------------------------------------------------------
def preset(name: str, scale: float = 1.0, steps: Optional[int] = None) -> Workload:
    """Named workloads.  ``scale`` shrinks node counts for quick runs."""
    if name == "sbm_n2000":
        return sbm_small(n0=max(8, int(2000 * scale)), new_per_step=max(1, int(100 * scale)),
                         insertions=max(1, int(300 * scale)), deletions=max(1, int(100 * scale)),
                         steps=steps or 10, cfg_id=1)
    if name == "chunglu_n1e5":
        return chung_lu(n0=max(64, int(100_000 * scale)), gamma=2.5, mean=16.0,
                        cap=min(2000.0, max(8.0, 2000.0 * scale ** 0.5)), steps=steps or 20, cfg_id=2)
    if name == "sbm_n1e6":
        return sbm_large(n0=max(256, int(1_000_000 * scale)), steps=steps or 10,
                         new_per_step=max(1, int(10_000 * scale)),
                         old_insertions=max(1, int(10_000 * scale)), cfg_id=3)
    if name == "chunglu_n4e6":
        return chung_lu(n0=max(256, int(4_000_000 * scale)), gamma=2.2, mean=16.0, cap=None,
                        steps=steps or 5, grow_frac=0.01, cfg_id=5)
    raise KeyError(name)
