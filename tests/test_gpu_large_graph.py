"""A graph of 9 million nodes: the row-pointer scans of the graph stage cover more than one
chunk of their block sums (4,096 blocks of 2,048 rows), so the carry between chunks is
exercised.  The merged graph must equal the oracle's A^(t+1) = pad(A^(t)) + Delta
(eq. adj_update) entry for entry, and the update must return orthonormal pairs.

The start is the ring graph, whose leading eigenvectors are known in closed form (the
constant vector and the first Fourier modes), so no eigensolve is needed to set it up.
"""
import sys

import numpy as np
import pytest

from oracle import grest_oracle as O
from paper_2603_19439_amd import grest as G

pytestmark = pytest.mark.gpu


def ring_csr(n):
    i = np.arange(n, dtype=np.int64)
    nb = np.stack([(i - 1) % n, (i + 1) % n], axis=1)
    nb.sort(axis=1)
    return np.arange(0, 2 * n + 1, 2, dtype=np.int64), nb.reshape(-1).astype(np.int32)


def test_graph_update_beyond_one_chunk_of_scan_block_sums():
    n = 9_000_000
    print(f"[gpu-case] ring graph n={n}, 3 appended nodes, 5 changes", flush=True)
    sys.stdout.flush()
    rp, col = ring_csr(n)
    t = 2.0 * np.pi * np.arange(n) / n
    X = np.stack([np.full(n, 1.0 / np.sqrt(n)), np.sqrt(2.0 / n) * np.cos(t), np.sqrt(2.0 / n) * np.sin(t),
                  np.sqrt(2.0 / n) * np.cos(2.0 * t)], axis=1)
    vals = np.array([2.0, 2.0 * np.cos(2 * np.pi / n), 2.0 * np.cos(2 * np.pi / n), 2.0 * np.cos(4 * np.pi / n)])
    st = G.State(rp, col, k=4, variant="g2", op="adj", precision="fp32", max_new=8)
    try:
        st.set_pairs(vals, X)
        ei = np.array([100, 200, 5, 7_000_000, n], dtype=np.int32)
        ej = np.array([101, 4_000_000, n, n + 1, n + 2], dtype=np.int32)
        sg = np.array([-1, 1, 1, 1, 1], dtype=np.int8)
        st.update(3, ei, ej, sg)
        st.sync()
        A = O.adjacency_from_csr(rp, col, n)
        Anew = O.updated_adjacency(O.pad_matrix(A, 3), O.assemble_delta(A, 3, ei, ej, sg))
        grp, gcol = st.graph()
        assert grp.shape == Anew.indptr.shape
        assert np.array_equal(grp, Anew.indptr), "row pointers differ"
        assert np.array_equal(gcol, Anew.indices), "column ids differ"
        _, Xn = st.get()
        assert Xn.shape == (n + 3, 4)
        assert np.abs(Xn.T @ Xn - np.eye(4)).max() < 1e-5
    finally:
        st.close()
