"""The update that allocates nothing (grest_update_noalloc) against grest_update.

Both entry points run the same kernels; the no-allocation variant takes the buffers sized
by the change list from a static device array instead of the state's own.  Two states
start from the same graph and the same pairs, one driven by each entry point, through two
updates in a row, the second with a smaller change list and fewer appended nodes; the
values, the tracked block and the stored graph must agree bit for bit after each.
"""
import sys

import numpy as np
import pytest

from oracle import grest_oracle as O
from paper_2603_19439_amd import grest as G
from paper_2603_19439_amd import workloads as W

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _two_updates(wl, Ls):
    """The workload's first update, then a smaller one: half of the second update's
    appended nodes and the first half of its changes among the nodes that then exist."""
    d1, d2 = wl.deltas[0], wl.deltas[1]
    n1 = wl.n0 + d1.n_new
    s2 = d2.n_new // 2
    keep = np.flatnonzero(d2.j < n1 + s2)
    keep = keep[: max(1, keep.size // 2)]
    i2, j2, g2 = d2.i[keep], d2.j[keep], d2.sign[keep]
    assert s2 < d1.n_new and keep.size < d1.n_changes
    om1 = W.omega(wl.cfg_id, 0, 1, d1.n_new, Ls) if Ls else None
    om2 = W.omega(wl.cfg_id, 0, 2, s2, Ls) if Ls and s2 > 0 else None
    return [(d1.n_new, d1.i, d1.j, d1.sign, om1), (s2, i2, j2, g2, om2)]


@pytest.mark.parametrize("case", ["rsvd_mixed", "rsvd_fp32_overlap", "g3_fp64", "rsvd_mixed_lowrank"])
def test_noalloc_update_matches_update(case):
    parts = case.split("_")
    variant, prec = parts[0], parts[1]
    overlap = "overlap" in parts
    proj = "lowrank" if "lowrank" in parts else "exact"
    if variant == "g3":
        wl = W.preset("sbm_n2000", scale=0.5, steps=2)
        k, L, P = 6, 0, 0
    else:
        wl = W.preset("sbm_n1e6", scale=0.01, steps=2)
        k, L, P = 8, 8, 8
    ups = _two_updates(wl, L + P if variant == "rsvd" else 0)
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, _ = O.leading_eigenpairs(A, k)
    cap_n = wl.n0 + sum(u[0] for u in ups) + 8
    cap_m = wl.col0.size + 2 * sum(u[1].size for u in ups) + 64
    outs = []
    for noalloc in (False, True):
        banner(f"no-alloc case={case} noalloc={noalloc} n0={wl.n0} S={[u[0] for u in ups]} "
               f"changes={[u[1].size for u in ups]}")
        st = G.State(wl.rowptr0, wl.col0, k=k, variant=variant, precision=prec, L=L, P=P,
                     max_new=max(u[0] for u in ups), node_capacity=cap_n, nnz_capacity=cap_m, proj=proj)
        st.set_pairs(th0, X0)
        st.set_overlap(overlap)
        seq = []
        for S, i, j, g, om in ups:
            st.update(S, i, j, g, om, noalloc=noalloc)
            st.sync()
            vals, X = st.get(np.float64)
            seq.append((vals, X) + (st.graph() if proj == "exact" else ()))
        outs.append(seq)
        st.close()
    for t, (a, b) in enumerate(zip(outs[0], outs[1])):
        for x, y in zip(a, b):
            assert x.shape == y.shape and np.array_equal(x, y), (case, t)


def test_noalloc_update_refuses_growth_and_keeps_the_state():
    """An update that would need a larger buffer is refused with EINVAL and nothing queued:
    more appended nodes than the node capacity, and a change list beyond the workspace."""
    wl = W.preset("sbm_n2000", scale=0.5, steps=1)
    k = 4
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, _ = O.leading_eigenpairs(A, k)
    d = wl.deltas[0]
    st = G.State(wl.rowptr0, wl.col0, k=k, variant="g3", precision="fp64", max_new=d.n_new,
                 node_capacity=wl.n0 + 1, nnz_capacity=wl.col0.size + 2 * d.n_changes)
    st.set_pairs(th0, X0)
    before = st.get()
    banner("no-alloc refusal: node capacity")
    with pytest.raises(G.GrestError) as e:
        st.update(d.n_new, d.i, d.j, d.sign, noalloc=True)
    assert e.value.status == G.EINVAL and "capacity" in str(e.value)
    banner("no-alloc refusal: change list beyond the workspace")
    big = (1 << 18) + 1
    ii = np.zeros(big, np.int32)
    with pytest.raises(G.GrestError) as e:
        st.update(0, ii, ii + 1, np.ones(big, np.int8), noalloc=True)
    assert e.value.status == G.EINVAL and "maximum" in str(e.value)
    st.sync()
    after = st.get()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    assert st.shape()[0] == wl.n0
    st.close()
