"""The seeded generators: determinism, validity of every update, and the shapes they promise."""
import numpy as np
import pytest

from paper_2603_19439_amd import workloads as W
from oracle import grest_oracle as O


def _valid_stream(wl, steps):
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    for d in wl.deltas[:steps]:
        D = O.assemble_delta(A, d.n_new, d.i, d.j, d.sign)  # raises on an invalid change list
        A = O.updated_adjacency(A, D)
    keys = wl.keys_at(steps)
    rp, col = W.csr_from_keys(A.shape[0], keys)
    assert np.array_equal(rp, A.indptr) and np.array_equal(col, A.indices)
    return A


@pytest.mark.parametrize("name,scale", [("sbm_n2000", 0.25), ("sbm_n1e6", 0.005),
                                        ("chunglu_n1e5", 0.02), ("chunglu_n4e6", 0.001)])
def test_streams_are_valid_and_deterministic(name, scale):
    a = W.preset(name, scale=scale, steps=3)
    b = W.preset(name, scale=scale, steps=3)
    assert np.array_equal(a.rowptr0, b.rowptr0) and np.array_equal(a.col0, b.col0)
    for da, db in zip(a.deltas, b.deltas):
        assert np.array_equal(da.i, db.i) and np.array_equal(da.sign, db.sign)
    _valid_stream(a, 3)


def test_sbm_small_shape():
    wl = W.preset("sbm_n2000", steps=2)
    deg = np.diff(wl.rowptr0)
    # 4 equal blocks of 500, p_in=0.05, p_out=0.005: mean degree 499*0.05 + 1500*0.005 = 32.45
    assert abs(deg.mean() - 32.45) < 1.0
    d = wl.deltas[0]
    assert d.n_new == 100
    old = d.j < wl.n0
    assert (d.sign[old] < 0).sum() == 100
    assert ((d.sign > 0) & old).sum() == 300


def test_sbm_large_shape():
    wl = W.preset("sbm_n1e6", scale=0.01, steps=1)
    deg = np.diff(wl.rowptr0)
    assert abs(deg.mean() - 20.0) < 1.0
    d = wl.deltas[0]
    assert d.n_new == 100 and (d.sign > 0).all()
    assert 300 < d.n_changes < 700  # ~4 per new node plus the old-old insertions


def test_chung_lu_shape_and_connectivity():
    from scipy.sparse.csgraph import connected_components
    wl = W.preset("chunglu_n1e5", scale=0.05, steps=1)
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    assert connected_components(A, directed=False)[0] == 1
    deg = np.diff(wl.rowptr0)
    assert 12 < deg.mean() < 18
    assert deg.max() > 10 * deg.mean()  # heavy tail


def test_omega_is_standard_normal_and_seeded():
    a = W.omega(3, 0, 1, 2000, 64)
    assert np.array_equal(a, W.omega(3, 0, 1, 2000, 64))
    assert abs(a.mean()) < 0.01 and abs(a.std() - 1) < 0.01


def test_sbm_expansion_structure():
    """The expansion SBM: the graph at t = 0 is induced by the first n0 ids, every update
    appends new_per_step nodes with insertions that touch a new node only, and the final
    graph's edge densities inside and across clusters match p_in and p_out."""
    N, k, p_in, p_out = 2000, 4, 0.05, 0.01
    cw = W.sbm_expansion(N=N, clusters=k, p_in=p_in, p_out=p_out, n0=1900, steps=10, new_per_step=10, graph_id=3)
    wl, lab = cw.workload, cw.labels
    assert wl.rowptr0.shape[0] == 1901 and lab.shape == (N,)
    n = 1900
    for d in wl.deltas:
        assert d.n_old == n and d.n_new == 10
        assert np.all(d.sign == 1) and np.all(d.i < d.j) and np.all(d.j >= n) and np.all(d.j < n + 10)
        n += 10
    keys = wl.keys_final
    i, j = keys // W.KEY_BASE, keys % W.KEY_BASE
    same = lab[i] == lab[j]
    sizes = np.bincount(lab, minlength=k)
    pairs_in = int((sizes * (sizes - 1) // 2).sum())
    pairs_out = N * (N - 1) // 2 - pairs_in
    for cnt, pairs, p in [(int(same.sum()), pairs_in, p_in), (int((~same).sum()), pairs_out, p_out)]:
        sd = np.sqrt(pairs * p * (1 - p))
        assert abs(cnt - pairs * p) <= 5 * sd, (cnt, pairs * p)
    # same seed, same stream
    again = W.sbm_expansion(N=N, clusters=k, p_in=p_in, p_out=p_out, n0=1900, steps=10, new_per_step=10, graph_id=3)
    assert np.array_equal(again.workload.keys_final, keys) and np.array_equal(again.labels, lab)
