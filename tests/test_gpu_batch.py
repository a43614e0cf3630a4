"""Batched updates of several graphs (grest_update_batch): the members' one-workgroup stages
(CholQR factors, small eigensolves) are launched once for all of them from device
descriptors.  Every graph must get exactly the results of its own updates run alone
(bitwise: the same kernels with the same arguments), whatever the other members are; a
member whose change list is invalid fails alone and leaves its state unchanged; one
batched graph is also checked against the FP64 oracle.
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


def _members():
    """Graphs of different sizes, K, variants, operators and precisions, with the exact
    initial pairs: a mix whose members take different kernel instances in each stage."""
    specs = [  # (n0, k, variant, op, prec, graph_id)
        (500, 4, "rsvd", "adj", "mixed", 21),
        (700, 8, "rsvd", "adj", "mixed", 22),
        (900, 16, "rsvd", "adj", "fp32", 23),
        (600, 6, "g3", "adj", "fp64", 24),
        (800, 8, "g2", "lap", "fp32", 25),
        (650, 24, "rsvd", "adj", "fp64", 26),
    ]
    out = []
    for n0, k, variant, op, prec, gid in specs:
        wl = W.sbm_small(n0=n0, new_per_step=20, insertions=60, deletions=20, steps=4, cfg_id=1, graph_id=gid)
        A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
        th, X, shift = O.leading_eigenpairs(A, k, op)
        vals = th if op == "adj" else shift - th  # the Laplacians' pairs are set as nu
        out.append(dict(wl=wl, k=k, variant=variant, op=op, prec=prec, th=th, vals=vals, X=X))
    return out


def _state(m):
    kw = dict(k=m["k"], variant=m["variant"], op=m["op"], precision=m["prec"])
    if m["variant"] == "rsvd":
        kw.update(L=m["k"], P=m["k"])
    if m["variant"] == "g3":
        kw.update(max_new=64)
    st = G.State(m["wl"].rowptr0, m["wl"].col0, **kw)
    st.set_pairs(m["vals"], m["X"])
    return st


def _omega(m, g, t, d):
    if m["variant"] != "rsvd" or d.n_new == 0:
        return None
    return W.omega(m["wl"].cfg_id, g, t + 1, d.n_new, 2 * m["k"])


def _alone(members, gids=None):
    """Every member's trajectory with its updates run one graph at a time (gids: the graph
    index each member's test matrices are drawn for; by default its position)."""
    ref = []
    for g, m in zip(gids or range(len(members)), members):
        st = _state(m)
        steps = []
        for t, d in enumerate(m["wl"].deltas):
            st.update_delta(d, _omega(m, g, t, d))
            st.sync()
            steps.append(st.get())
        ref.append(steps)
        st.close()
    return ref


def test_batch_matches_each_graph_alone():
    members = _members()
    banner(f"batch of {len(members)}: references one graph at a time")
    ref = _alone(members)
    states = [_state(m) for m in members]
    steps = len(members[0]["wl"].deltas)
    for t in range(steps):
        banner(f"batch step {t + 1}")
        ups = []
        for g, (m, st) in enumerate(zip(members, states)):
            d = m["wl"].deltas[t]
            ups.append((st, d.n_new, d.i, d.j, d.sign, _omega(m, g, t, d)))
        status = G.update_batch(ups)
        assert status == [G.OK] * len(members), status
        for g, st in enumerate(states):
            st.sync()
            vals, X = st.get()
            rv, rX = ref[g][t]
            assert np.array_equal(vals, rv), (g, t)
            assert np.array_equal(X, rX), (g, t)
    for st in states:
        st.close()


def test_batch_of_one_and_a_subset_in_any_order():
    members = _members()[:4]
    ref = _alone(members)
    states = [_state(m) for m in members]
    steps = len(members[0]["wl"].deltas)
    for t in range(steps):
        # step t batches a rotating subset (one member alone at t = 0), the rest alone
        order = list(range(len(members)))
        order = order[t % len(order):] + order[:t % len(order)]
        batched = order[: max(1, t)]
        banner(f"subset step {t + 1}: batched {batched}")
        ups = []
        for g in batched:
            d = members[g]["wl"].deltas[t]
            ups.append((states[g], d.n_new, d.i, d.j, d.sign, _omega(members[g], g, t, d)))
        assert G.update_batch(ups) == [G.OK] * len(batched)
        for g in order[len(batched):]:
            d = members[g]["wl"].deltas[t]
            states[g].update_delta(d, _omega(members[g], g, t, d))
        for g, st in enumerate(states):
            st.sync()
            vals, X = st.get()
            assert np.array_equal(vals, ref[g][t][0]) and np.array_equal(X, ref[g][t][1]), (g, t)
    for st in states:
        st.close()


def test_invalid_member_fails_alone():
    members = _members()[:3]
    states = [_state(m) for m in members]
    before = [st.get() for st in states]
    ups = []
    for g, (m, st) in enumerate(zip(members, states)):
        d = m["wl"].deltas[0]
        i, j, sign = d.i, d.j, d.sign
        if g == 1:  # an insertion of an existing edge: refused by the device validation
            wl = m["wl"]
            r = 0
            c = int(wl.col0[wl.rowptr0[r]])
            i = np.concatenate([i, np.array([min(r, c)], np.int32)])
            j = np.concatenate([j, np.array([max(r, c)], np.int32)])
            sign = np.concatenate([sign, np.array([1], np.int8)])
        ups.append((st, d.n_new, i, j, sign, _omega(m, g, 0, d)))
    banner("batch with an invalid member")
    with pytest.raises(G.GrestError) as e:
        G.update_batch(ups)
    assert e.value.status == G.EINVAL
    ref = _alone([members[0], members[2]], gids=[0, 2])
    states[1].sync()
    vals, X = states[1].get()
    assert np.array_equal(vals, before[1][0]) and np.array_equal(X, before[1][1])
    for g, r in ((0, ref[0][0]), (2, ref[1][0])):
        states[g].sync()
        vals, X = states[g].get()
        assert np.array_equal(vals, r[0]) and np.array_equal(X, r[1]), g
    for st in states:
        st.close()


def test_batched_graph_matches_oracle():
    m = _members()[1]  # RSVD, mixed precision, K = 8
    others = _members()[2:4]
    states = [_state(x) for x in [m] + others]
    wl, k = m["wl"], m["k"]
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    theta, Xo = m["th"].copy(), m["X"].copy()
    r = None
    for t, d in enumerate(wl.deltas):
        ups = []
        for g, (x, st) in enumerate(zip([m] + others, states)):
            dd = x["wl"].deltas[t]
            ups.append((st, dd.n_new, dd.i, dd.j, dd.sign, _omega(x, g, t, dd)))
        assert G.update_batch(ups) == [G.OK] * 3
        r = O.grest_step(A, Xo, theta, d.n_new, d.i, d.j, d.sign, k, variant=O.RSVD, L=k, Omega=_omega(m, 0, t, d))
        A, Xo, theta = r.A, r.X, r.theta
    states[0].sync()
    vals, X = states[0].get()
    # the gate covers the prefix separated from the rest of the oracle's Ritz spectrum
    th_all = np.linalg.eigvalsh(r.H)
    keys = np.abs(th_all[O.select(th_all, th_all.size, O.which_for("adj"))])
    kstar = M.gap_prefix(keys, k, 1e-3)
    e = M.eig_rel_error(vals[:kstar], theta[:kstar])
    s = M.subspace_sine(X[:, :kstar], Xo[:, :kstar]) if kstar > 0 else 0.0
    banner(f"batched graph vs oracle: k*={kstar} e_lambda {e:.2e} sine {s:.2e}")
    assert e <= 1e-3 and s <= 1e-3
    for st in states:
        st.close()
