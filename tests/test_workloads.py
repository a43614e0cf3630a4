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
