"""Batched execution of many graphs through the serving entry points (grest_server_*).

The server runs the single-graph update for several graphs on several lanes (host
threads with their own streams).  What it must guarantee, and what is checked here:
a graph's result does not depend on the other graphs in the mix or on the lane
interleaving (bitwise equal to the same updates run alone), per-graph order is kept,
an invalid request fails alone and leaves its graph unchanged, admission limits are
enforced, and completion records carry consistent time stamps.  The numerical quality
of each update is the parity suite's business; one graph here is also checked
against the FP64 oracle.
"""
import sys

import numpy as np
import pytest

from oracle import grest_oracle as O
from paper_2603_19439_amd import grest as G
from paper_2603_19439_amd import metrics as M
from paper_2603_19439_amd import workloads as W

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _graphs(count, n0=600, steps=4, new=20):
    """Small SBM graphs with different seeds and K, with the exact initial pairs."""
    out = []
    for g in range(count):
        wl = W.sbm_small(n0=n0 + 40 * g, new_per_step=new, insertions=60, deletions=20, steps=steps, cfg_id=1,
                         graph_id=10 + g)
        k = (4, 6, 8)[g % 3]
        A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
        th, X, _ = O.leading_eigenpairs(A, k)
        out.append((wl, k, th, X))
    return out


def _new_state(wl, k, th, X, prec):
    st = G.State(wl.rowptr0, wl.col0, k=k, variant="rsvd", precision=prec, L=k, P=k)
    st.set_pairs(th, X)
    return st


def _omega(wl, g, t, d, k):
    return W.omega(wl.cfg_id, g, t + 1, d.n_new, 2 * k) if d.n_new > 0 else None


@pytest.mark.parametrize("prec,batch", [("fp64", 1), ("mixed", 1), ("mixed", 3), ("fp64", 2)])
def test_results_do_not_depend_on_the_mix(prec, batch):
    """Also with lanes that run batches (grest_server_create_batched): a graph's updates
    go through grest_update_batch with whatever other graphs were runnable."""
    graphs = _graphs(3 if batch == 1 else 5)
    # reference: every graph alone, updates driven directly
    ref = []
    for g, (wl, k, th, X) in enumerate(graphs):
        banner(f"serving reference graph {g} prec={prec} n0={wl.n0} k={k}")
        st = _new_state(wl, k, th, X, prec)
        for t, d in enumerate(wl.deltas):
            st.update_delta(d, _omega(wl, g, t, d, k))
        st.sync()
        ref.append(st.get())
        st.close()
    # the same updates interleaved over two lanes
    banner(f"serving mix prec={prec} batch={batch}")
    sv = G.Server(lanes=2, batch=batch)
    states = [_new_state(wl, k, th, X, prec) for (wl, k, th, X) in graphs]
    ids = [sv.attach(st) for st in states]
    tag = 0
    steps = len(graphs[0][0].deltas)
    for t in range(steps):
        for g, (wl, k, th, X) in enumerate(graphs):
            d = wl.deltas[t]
            rc = sv.submit(ids[g], d.n_new, d.i, d.j, d.sign, _omega(wl, g, t, d, k), tag=1000 * g + t)
            assert rc == G.OK, rc
            tag += 1
    sv.drain()
    tags, status, ts, td = sv.poll(1024)
    assert tags.size == tag and np.all(status == G.OK), (tags, status)
    assert np.all(td >= ts)
    # per-graph completion order follows submission order
    for g in range(len(graphs)):
        mine = [int(x) % 1000 for x in tags if int(x) // 1000 == g]
        assert mine == sorted(mine), mine
    sv.close()
    for g, st in enumerate(states):
        vals, X = st.get()
        assert np.array_equal(vals, ref[g][0]) and np.array_equal(X, ref[g][1]), f"graph {g} differs"
        st.close()


def test_served_graph_matches_oracle():
    (wl, k, th, X), = _graphs(1)
    banner(f"serving vs oracle n0={wl.n0} k={k}")
    sv = G.Server(lanes=3)
    st = _new_state(wl, k, th, X, "fp64")
    gid = sv.attach(st)
    for t, d in enumerate(wl.deltas):
        assert sv.submit(gid, d.n_new, d.i, d.j, d.sign, _omega(wl, 0, t, d, k), tag=t) == G.OK
    sv.drain()
    _, status, _, _ = sv.poll(64)
    assert np.all(status == G.OK)
    sv.close()
    A, Xo, tho = O.adjacency_from_csr(wl.rowptr0, wl.col0), X, th
    for t, d in enumerate(wl.deltas):
        r = O.grest_step(A, Xo, tho, d.n_new, d.i, d.j, d.sign, k, variant=O.RSVD, L=k,
                         Omega=_omega(wl, 0, t, d, k))
        A, Xo, tho = r.A, r.X, r.theta
    vals, Xg = st.get()
    # the gate covers the prefix separated from the rest of the oracle's Ritz spectrum (all
    # of its projected matrix's values, not only the K tracked ones)
    th_all = np.linalg.eigvalsh(r.H)
    keys = np.abs(th_all[O.select(th_all, th_all.size, O.which_for("adj"))])
    kk = M.gap_prefix(keys, k, 1e-3)
    assert M.eig_rel_error(vals[:kk], tho[:kk]) <= 1e-10
    if kk > 0:
        assert M.subspace_sine(Xg[:, :kk], Xo[:, :kk]) <= 1e-8
    st.close()


def test_invalid_request_fails_alone():
    (wl, k, th, X), = _graphs(1)
    banner("serving invalid request")
    # reference: only the valid first update
    st_ref = _new_state(wl, k, th, X, "fp64")
    d0 = wl.deltas[0]
    st_ref.update_delta(d0, _omega(wl, 0, 0, d0, k))
    st_ref.sync()
    ref = st_ref.get()
    st_ref.close()
    sv = G.Server(lanes=1)
    st = _new_state(wl, k, th, X, "fp64")
    gid = sv.attach(st)
    # an insertion of an existing edge passes the host checks and fails on the device
    i0 = int(np.repeat(np.arange(wl.n0), np.diff(wl.rowptr0))[0])
    j0 = int(wl.col0[0])
    a, b = min(i0, j0), max(i0, j0)
    assert sv.submit(gid, 0, np.array([a]), np.array([b]), np.array([1], np.int8), None, tag=1) == G.OK
    assert sv.submit(gid, d0.n_new, d0.i, d0.j, d0.sign, _omega(wl, 0, 0, d0, k), tag=2) == G.OK
    # a host-detectable error is refused at submission
    assert sv.submit(gid, 0, np.array([3]), np.array([3]), np.array([1], np.int8), None, tag=3) == G.EINVAL
    sv.drain()
    tags, status, _, _ = sv.poll(16)
    assert list(tags) == [1, 2] and status[0] == G.EINVAL and status[1] == G.OK, (tags, status)
    sv.close()
    vals, Xg = st.get()
    assert np.array_equal(vals, ref[0]) and np.array_equal(Xg, ref[1])
    st.close()


def test_admission_limits():
    (wl, k, th, X), = _graphs(1)
    banner("serving admission: budget below one state")
    st = _new_state(wl, k, th, X, "fp64")
    assert st.memory() > 0
    sv = G.Server(lanes=1, hbm_budget_bytes=1)
    with pytest.raises(G.GrestError) as e:
        sv.attach(st)
    assert e.value.status == G.EAGAIN
    sv.close()
    st.close()


def _fresh_insertions(wl, count, seed, avoid=()):
    """`count` insertions among the initial nodes: pairs that are not edges of the initial
    graph and do not appear in the change lists `avoid` (so they stay valid whatever of
    those runs first)."""
    n = wl.n0
    taken = set()
    for r in range(n):
        for c in wl.col0[wl.rowptr0[r]:wl.rowptr0[r + 1]]:
            taken.add((r, int(c)))
    for d in avoid:
        taken.update(zip(d.i.tolist(), d.j.tolist()))
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        a, b = sorted(rng.integers(0, n, 2).tolist())
        if a < b and (a, b) not in taken:
            taken.add((a, b))
            out.append((a, b))
    i, j = (np.array(x, dtype=np.int32) for x in zip(*out))
    return i, j, np.ones(count, dtype=np.int8)


def test_admission_by_memory_and_detach():
    """Admission by device memory, deterministic: the server reserves each graph's
    footprint plus the growth of its queued requests.  A request that would outgrow the
    state's node capacity is refused while the budget is tight, a request within the
    capacities is admitted, and after a detach releases another graph's reservation the
    growing request is admitted and runs; the reservation then equals the actual
    footprint of the attached states and never exceeds the budget."""
    graphs = _graphs(2, n0=600)
    (wa, ka, tha, Xa), (wb, kb, thb, Xb) = graphs
    banner("serving admission by memory")
    # A: node capacity exactly its node count (+1), so appended nodes force a reallocation
    sa = G.State(wa.rowptr0, wa.col0, k=ka, variant="rsvd", precision="fp64", L=ka, P=ka,
                 node_capacity=wa.n0 + 1)
    sa.set_pairs(tha, Xa)
    sb = G.State(wb.rowptr0, wb.col0, k=kb, variant="rsvd", precision="fp64", L=kb, P=kb,
                 node_capacity=4 * wb.n0)
    sb.set_pairs(thb, Xb)
    ma, mb = sa.memory(), sb.memory()
    budget = ma + mb + 4096
    sv = G.Server(lanes=2, hbm_budget_bytes=budget)
    ga, gb = sv.attach(sa), sv.attach(sb)
    assert sv.memory() == (ma + mb, budget)
    d0 = wa.deltas[0]
    om0 = _omega(wa, 0, 0, d0, ka)
    assert d0.n_new > 1
    # growth of A's node buffers does not fit: refused, nothing reserved
    assert sv.submit(ga, d0.n_new, d0.i, d0.j, d0.sign, om0, tag=1) == G.EAGAIN
    assert sv.memory()[0] == ma + mb
    # a request within A's capacities is admitted and runs
    i1, j1, s1 = _fresh_insertions(wa, 40, 1, avoid=[d0])
    assert sv.submit(ga, 0, i1, j1, s1, None, tag=2) == G.OK
    sv.drain()
    tags, status, _, _ = sv.poll(16)
    assert list(tags) == [2] and list(status) == [G.OK]
    assert sv.memory()[0] == sa.memory() + mb <= budget
    # detach B: its reservation is released and A's growing request now fits
    assert sv.detach(gb) == G.OK
    assert sv.memory()[0] == sa.memory()
    assert sv.detach(gb) == G.EINVAL
    assert sv.submit(gb, 0, i1[:1], j1[:1], s1[:1], None, tag=9) == G.EINVAL
    rc = sv.submit(ga, d0.n_new, d0.i, d0.j, d0.sign, om0, tag=3)
    assert rc == G.OK, rc
    assert sv.memory()[0] <= budget
    sv.drain()
    tags, status, _, _ = sv.poll(16)
    assert list(tags) == [3] and list(status) == [G.OK]
    reserved = sv.memory()[0]
    assert reserved == sa.memory() and reserved <= budget and sa.memory() > ma
    assert sa.shape()[0] == wa.n0 + d0.n_new
    sv.close()
    # the detached state is usable directly, and so is A after the server is gone
    db = wb.deltas[0]
    sb.update_delta(db, _omega(wb, 1, 0, db, kb))
    sb.sync()
    class _Pairs:  # the insertions already applied, to be avoided by the last one
        i, j = i1, j1
    sa.update(0, *_fresh_insertions(wa, 10, 2, avoid=[d0, _Pairs]))
    sa.sync()
    sa.close()
    sb.close()


@pytest.mark.parametrize("graph_id,requests", [(16, 4), (14, 20)])
def test_serving_graph_updates_report_no_numerical_status(graph_id, requests):
    """Graphs of the serving mix on which the small eigensolver once read an unset entry
    of its LU factor (regression): every update must finish with status OK."""
    sg = W.serving_graph(graph_id, requests)
    wl = sg.workload
    banner(f"serving graph {graph_id} ({sg.family}, n0={wl.n0}, k={sg.k}) for {requests} requests")
    n_fin = wl.n0 + sum(d.n_new for d in wl.deltas) + 1
    nnz = int(wl.col0.size + 2 * sum(d.n_changes for d in wl.deltas) + 1024)
    st = G.State(wl.rowptr0, wl.col0, k=sg.k, variant="rsvd", precision="mixed", L=sg.k, P=sg.k,
                 node_capacity=n_fin, nnz_capacity=nnz)
    st.init_pairs(iterations=20, seed=graph_id)
    for t, d in enumerate(wl.deltas):
        st.update_delta(d, W.omega(4, graph_id, t + 1, d.n_new, 2 * sg.k) if d.n_new > 0 else None)
        st.sync()  # raises on a non-OK status
    vals, X = st.get()
    assert np.all(np.isfinite(vals)) and np.all(np.isfinite(X))
    assert M.orthonormality(X) <= 1e-5
    st.close()


def test_restart_policy_inside_served_updates():
    """States with a restart policy served over two lanes: the recomputations happen inside
    the lanes' updates, after the same updates as when each graph is driven alone, and
    the results are bitwise those of the graph alone."""
    graphs = _graphs(3, steps=4)

    def policy_state(g, wl, k, th, X):
        st = _new_state(wl, k, th, X, "fp64")
        st.set_restart(0.0, 0.0, check_every=1, min_gap=2, iterations=20, seed=7 + g)
        return st

    ref = []
    for g, (wl, k, th, X) in enumerate(graphs):
        banner(f"restart policy alone graph {g}")
        st = policy_state(g, wl, k, th, X)
        for t, d in enumerate(wl.deltas):
            st.update_delta(d, _omega(wl, g, t, d, k))
        st.sync()
        ref.append((st.get(), st.restart_stats()[0]))
        st.close()
    banner("restart policy served")
    sv = G.Server(lanes=2)
    states = [policy_state(g, wl, k, th, X) for g, (wl, k, th, X) in enumerate(graphs)]
    ids = [sv.attach(st) for st in states]
    for t in range(4):
        for g, (wl, k, th, X) in enumerate(graphs):
            d = wl.deltas[t]
            assert sv.submit(ids[g], d.n_new, d.i, d.j, d.sign, _omega(wl, g, t, d, k), tag=1000 * g + t) == G.OK
    sv.drain()
    tags, status, _, _ = sv.poll(1024)
    assert tags.size == 12 and np.all(status == G.OK), status
    sv.close()
    for g, st in enumerate(states):
        (vr, Xr), nr = ref[g]
        vals, X = st.get()
        assert nr == 2 and st.restart_stats()[0] == nr
        assert np.array_equal(vals, vr) and np.array_equal(X, Xr), f"graph {g} differs"
        st.close()


def test_graph_free_lowrank_states_served():
    """Low-rank states that released their graphs (the truncated form keeps Delta alone)
    are admitted with the footprint they have after the release and served with results
    bitwise those of each graph alone.  Their node capacity covers every update, so the
    requests need no growth and fit a budget of exactly the attached footprints."""
    graphs = _graphs(3, steps=3)

    def lowrank_state(wl, k, th, X):
        st = G.State(wl.rowptr0, wl.col0, k=k, variant="rsvd", precision="mixed", L=k, P=k, proj="lowrank",
                     node_capacity=wl.n_at(3) + 1)
        st.set_pairs(th, X)
        before = st.memory()
        st.release_graph()
        assert st.memory() < before
        return st

    ref = []
    for g, (wl, k, th, X) in enumerate(graphs):
        banner(f"graph-free low-rank alone graph {g}")
        st = lowrank_state(wl, k, th, X)
        for t, d in enumerate(wl.deltas):
            st.update_delta(d, _omega(wl, g, t, d, k))
        st.sync()
        ref.append(st.get())
        st.close()
    banner("graph-free low-rank served")
    states = [lowrank_state(wl, k, th, X) for (wl, k, th, X) in graphs]
    sv = G.Server(lanes=2, hbm_budget_bytes=sum(st.memory() for st in states))
    ids = [sv.attach(st) for st in states]
    for t in range(3):
        for g, (wl, k, th, X) in enumerate(graphs):
            d = wl.deltas[t]
            assert sv.submit(ids[g], d.n_new, d.i, d.j, d.sign, _omega(wl, g, t, d, k), tag=1000 * g + t) == G.OK
    sv.drain()
    tags, status, _, _ = sv.poll(1024)
    assert tags.size == 9 and np.all(status == G.OK), status
    sv.close()
    for g, st in enumerate(states):
        vals, X = st.get()
        assert np.array_equal(vals, ref[g][0]) and np.array_equal(X, ref[g][1]), f"graph {g} differs"
        st.close()
