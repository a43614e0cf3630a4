"""Parity of the HIP path (through the C interface) with the FP64 oracle.

Both sides get the same seeded inputs: the same graph, the same change lists, the
same Gaussian test matrix and the same initial pairs (computed here on the host by
dense eigh / ARPACK, never by the GPU).  Tolerances are the ones the update is
judged by: eigenvalue relative error <= 1e-10 in FP64, <= 1e-5 in FP32 and
<= 1e-3 with BF16 products, and subspace sine <= 1e-3 on the part of the tracked
set that is separated from the rest by a relative gap of at least 1e-3.
"""
import sys

import numpy as np
import pytest

from oracle import grest_oracle as O
from paper_2603_19439_amd import grest as G
from paper_2603_19439_amd import metrics as M
from paper_2603_19439_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_EIG = {"fp64": 1e-10, "fp32": 1e-5, "mixed": 1e-3}
TOL_SINE = {"fp64": 1e-8, "fp32": 1e-3, "mixed": 1e-3}
TOL_ORTH = {"fp64": 1e-12, "fp32": 1e-5, "mixed": 1e-5}


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def oracle_values(r: O.StepResult, op: str, proj: str = "exact"):
    """The values the method reports: Ritz values of the projected matrix.  For the
    Laplacians nu = shift - theta, evaluated as the quadratic form x^T L x of the Ritz
    vectors for the exact form (the same number, without cancellation against the shift);
    the truncated form's Ritz values are those of its own projected matrix, which the
    quadratic form on the true L does not give."""
    if op == "adj":
        return r.theta
    return r.nu if proj == "lowrank" else r.nu_rq


def check_step(st, r, op, prec, k, label, proj="exact"):
    vals, X = st.get()
    ref = oracle_values(r, op, proj)
    # the gate covers the prefix k* <= K of the tracked set that is separated from the
    # rest by a gap >= 1e-3 of the scale: |theta_1| for the adjacency, the largest tracked
    # nu for the Laplacians
    th_all = np.linalg.eigvalsh(r.H)
    order = O.select(th_all, th_all.size, O.which_for(op))
    if op == "adj":
        kk = M.gap_prefix(np.abs(th_all[order]), k, 1e-3)
    else:  # gaps between the nu = shift - theta, relative to the tracked nu's scale (not the shift)
        nu = r.shift - th_all[order]
        kk = M.gap_prefix(nu, k, 1e-3, scale=max(float(np.abs(nu[:k]).max()), 1e-300))
    if op == "adj":
        e = M.eig_rel_error(vals[:kk], ref[:kk])
    else:
        # Laplacians: relative error on nu without the trivial pair, which is compared in
        # absolute terms against the scale of the tracked spectrum
        e = M.eig_rel_error(vals[1:kk], ref[1:kk]) if kk > 1 else 0.0
        assert abs(vals[0] - ref[0]) <= 10 * TOL_EIG[prec] * max(1.0, np.abs(ref).max()), (label, vals[0], ref[0])
    sine = M.subspace_sine(X[:, :kk], r.X[:, :kk]) if kk > 0 else 0.0
    orth = M.orthonormality(X)
    banner(f"{label}: e_lambda={e:.3e} sine(k*={kk})={sine:.3e} orth={orth:.3e}")
    assert e <= TOL_EIG[prec], (label, e)
    assert sine <= TOL_SINE[prec], (label, sine)
    assert orth <= TOL_ORTH[prec], (label, orth)
    return vals, X


def run_trajectory(wl, k, variant, op, prec, steps, L=0, P=0, max_new=0, single_step=False, check_graph=True,
                   proj="exact"):
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, shift0 = O.leading_eigenpairs(A, k, op)
    vals0 = th0 if op == "adj" else shift0 - th0
    st = G.State(wl.rowptr0, wl.col0, k=k, variant=variant, op=op, precision=prec, L=L, P=P, max_new=max_new,
                 proj=proj)
    st.set_pairs(vals0, X0)
    Xo, tho = X0, th0
    for t, d in enumerate(wl.deltas[:steps]):
        om = W.omega(wl.cfg_id, 0, t + 1, d.n_new, L + P) if variant == "rsvd" and d.n_new > 0 else None
        banner(f"{wl.name} step {t + 1} variant={variant} op={op} prec={prec} n={A.shape[0]} S={d.n_new} "
               f"changes={d.n_changes}")
        st.update_delta(d, om)
        st.sync()
        r = O.grest_step(A, Xo, tho, d.n_new, d.i, d.j, d.sign, k, variant=variant, op=op, L=L or None, Omega=om,
                         proj=proj)
        if check_graph:
            rp, col = st.graph()
            assert np.array_equal(rp, r.A.indptr) and np.array_equal(col, r.A.indices), "graph update differs"
        vals, X = check_step(st, r, op, prec, k, f"step {t + 1}", proj)
        A = r.A
        if single_step:  # feed the oracle's state back to the GPU
            st.set_pairs(oracle_values(r, op, proj), r.X)
        Xo, tho = r.X, r.theta
    st.close()


# ------------------------------------------------------------------------------------
# end-to-end parity
# ------------------------------------------------------------------------------------
def test_sbm_n2000_fp64_g3_full_trajectory():
    """Plain method in FP64: SBM n0=2000 (4 blocks, 0.05/0.005), K=8, 10 steps of 100 new
    nodes + 300 insertions + 100 deletions, G-REST3."""
    wl = W.preset("sbm_n2000")
    run_trajectory(wl, 8, "g3", "adj", "fp64", 10, max_new=100)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_sbm_small_g2(prec):
    wl = W.preset("sbm_n2000", scale=0.5, steps=3)
    run_trajectory(wl, 8, "g2", "adj", prec, 3)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_sbm_large_shape_rsvd(prec):
    """Dirichlet SBM scaled to n0=20000 with RSVD (L=P=16), K=16."""
    wl = W.preset("sbm_n1e6", scale=0.02, steps=3)
    run_trajectory(wl, 16, "rsvd", "adj", prec, 3, L=16, P=16)


def test_chunglu_n1e5_normalized_laplacian_k32_fp32_full_size():
    """The normalised-Laplacian workload at its full size: Chung-Lu n0 = 1e5 (Pareto
    exponent 2.5, mean 16, cap 2000), K = 32, 20 steps of 0.5 % insertions and 0.2 %
    deletions, FP32, step by step against the oracle's trajectory (graph and pairs)."""
    wl = W.preset("chunglu_n1e5", steps=20)
    run_trajectory(wl, 32, "g2", "nlap", "fp32", 20)


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_sbm_headline_width_rsvd_k32(prec):
    """The headline's shape at n0=20000: Dirichlet SBM, K=32, RSVD with L=P=32, so the
    basis is 96 wide (the widths the large runs use in every product kernel)."""
    wl = W.preset("sbm_n1e6", scale=0.02, steps=2)
    run_trajectory(wl, 32, "rsvd", "adj", prec, 2, L=32, P=32)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_chunglu_normalized_laplacian(prec):
    """Chung-Lu (gamma 2.5, mean 16) with edge churn, normalised Laplacian, K=16, G-REST2."""
    wl = W.preset("chunglu_n1e5", scale=0.05, steps=3)
    run_trajectory(wl, 16, "g2", "nlap", prec, 3, single_step=True)


@pytest.mark.parametrize("op", ["lap", "nlap"])
def test_laplacians_with_growth_fp64(op):
    """Chung-Lu with node growth (gamma 2.2), both Laplacians, G-REST3 and RSVD."""
    wl = W.preset("chunglu_n4e6", scale=0.001, steps=2)
    run_trajectory(wl, 8, "g3", op, "fp64", 2, max_new=64)
    run_trajectory(wl, 8, "rsvd", op, "fp64", 2, L=8, P=8)


def _hub_workload(n0=3000, steps=2, hub_ins=400, hub_del=150, seed=5, new_hub=False):
    """SBM graph whose updates give one node hundreds of changes at once (a row of Delta
    longer than the 128 entries the row-split product takes), besides appended nodes and
    scattered changes: the shape of a power-law graph whose hub gains and loses many edges
    in one update.  With new_hub the node is the first appended one (insertions only)."""
    wl = W.sbm_small(n0=n0, new_per_step=30, insertions=200, deletions=60, steps=steps, cfg_id=1, graph_id=77)
    rng = np.random.default_rng(seed)
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    deltas = []
    for d in wl.deltas:
        n = A.shape[0]
        taken = set(zip(d.i.tolist(), d.j.tolist()))
        hub = n if new_hub else int(rng.integers(0, n))
        nbrs = set() if new_hub else set(A.indices[A.indptr[hub]:A.indptr[hub + 1]].tolist())
        pair = lambda v: (min(hub, v), max(hub, v))  # noqa: E731
        ins = [v for v in rng.permutation(n).tolist() if v != hub and v not in nbrs and pair(v) not in taken]
        dels = [v for v in rng.permutation(sorted(nbrs)).tolist() if pair(v) not in taken]
        ins, dels = ins[:hub_ins], ([] if new_hub else dels[:hub_del])
        ei = np.concatenate([d.i, [pair(v)[0] for v in ins + dels]]).astype(np.int64)
        ej = np.concatenate([d.j, [pair(v)[1] for v in ins + dels]]).astype(np.int64)
        sg = np.concatenate([d.sign, np.r_[np.ones(len(ins)), -np.ones(len(dels))]]).astype(np.int8)
        nd = W.Delta(n_old=n, n_new=d.n_new, i=ei, j=ej, sign=sg)
        deltas.append(nd)
        A = O.updated_adjacency(A, O.assemble_delta(A, nd.n_new, nd.i, nd.j, nd.sign))
    return W.Workload(name="sbm_hub", cfg_id=1, n0=wl.n0, rowptr0=wl.rowptr0, col0=wl.col0, deltas=deltas)


@pytest.mark.parametrize("op,variant,prec,new_hub", [("adj", "rsvd", "mixed", False), ("lap", "rsvd", "fp64", False),
                                                     ("adj", "g2", "fp32", False), ("adj", "rsvd", "fp64", True),
                                                     ("lap", "rsvd", "mixed", True)])
def test_heavy_delta_rows(op, variant, prec, new_hub):
    """A node gains 400 edges (and, if it is an old node, loses some of its own) in one
    update: its row of Delta goes to the workgroup-per-row path of Delta_1 Xbar (Prop. 3)
    and, for an appended node, of the sketch's Delta_2^T M (Sec. 3.5); the trajectory
    against the oracle's."""
    wl = _hub_workload(new_hub=new_hub)
    assert max(np.bincount(np.concatenate([d.i, d.j])).max() for d in wl.deltas) > 128
    kw = dict(L=8, P=8) if variant == "rsvd" else {}
    run_trajectory(wl, 8, variant, op, prec, 2, **kw)


def test_lowrank_projection_sbm_n2000_fp64_g3():
    """The paper's own form of the projected matrix (eq. RR_eigen_graph_upd_main3):
    H = Z^T Xbar Theta Xbar^T Z + Z^T Delta Z with the previous Ritz values, no product with
    the whole graph.  SBM n0 = 2000, K = 8, G-REST3, 5 steps, against the oracle's lowrank
    form on the same inputs."""
    wl = W.preset("sbm_n2000", steps=5)
    run_trajectory(wl, 8, "g3", "adj", "fp64", 5, max_new=100, proj="lowrank")


@pytest.mark.parametrize("variant,prec", [("g3", "fp64"), ("rsvd", "fp64"), ("rsvd", "mixed")])
def test_lowrank_projection_laplacian(variant, prec):
    """The low-rank form for the shifted combinatorial Laplacian T = alpha I - L (Sec. 4.2
    with eq. RR_eigen_graph_upd_main3): Chung-Lu with node growth and a hub, 2 steps,
    against the oracle's low-rank form (T's change from the degree changes and the shift)."""
    wl = W.preset("chunglu_n4e6", scale=0.001, steps=2)
    kw = dict(max_new=64) if variant == "g3" else dict(L=8, P=8)
    run_trajectory(wl, 8, variant, "lap", prec, 2, proj="lowrank", **kw)


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_lowrank_projection_sbm_large_shape_rsvd(prec):
    """The low-rank form with RSVD on the n = 1e6 SBM shape at 2 % scale (K = 16, L = P = 16)."""
    wl = W.preset("sbm_n1e6", scale=0.02, steps=3)
    run_trajectory(wl, 16, "rsvd", "adj", prec, 3, L=16, P=16, proj="lowrank")


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_lowrank_headline_width_graph_free(prec):
    """The low-rank form at the headline's width (K = 32, L = P = 32: a 96-wide basis) on
    the n = 1e6 SBM shape at 2 % scale, by a state that has released its graph and runs in
    the overlap mode, against the oracle's low-rank trajectory."""
    wl = W.preset("sbm_n1e6", scale=0.02, steps=2)
    k, L, P = 32, 32, 32
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, _ = O.leading_eigenpairs(A, k, "adj")
    st = G.State(wl.rowptr0, wl.col0, k=k, variant="rsvd", op="adj", precision=prec, L=L, P=P, proj="lowrank")
    st.set_pairs(th0, X0)
    st.release_graph()
    st.set_overlap(True)
    Xo, tho = X0, th0
    for t, d in enumerate(wl.deltas[:2]):
        om = W.omega(wl.cfg_id, 0, t + 1, d.n_new, L + P) if d.n_new > 0 else None
        banner(f"lowrank headline width step {t + 1} prec={prec} S={d.n_new} changes={d.n_changes}")
        st.update_delta(d, om)
        st.sync()
        r = O.grest_step(A, Xo, tho, d.n_new, d.i, d.j, d.sign, k, variant="rsvd", op="adj", L=L, Omega=om,
                         proj="lowrank")
        check_step(st, r, "adj", prec, k, f"step {t + 1}")
        A, Xo, tho = r.A, r.X, r.theta
    st.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lowrank_without_stored_graph(prec):
    """A low-rank state that has released its graph keeps Delta alone (the memory of
    eq. RR_eigen_graph_upd_main3's form): its pairs equal, bit for bit, those of a low-rank
    state that keeps the graph; it holds less device memory; the calls that need the
    graph refuse; a pair listed twice is still rejected, the state unchanged."""
    import torch
    wl = W.preset("sbm_n1e6", scale=0.02, steps=3)
    k, L, P = 16, 16, 16
    banner(f"lowrank without stored graph prec={prec}")
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, _ = O.leading_eigenpairs(A, k, "adj")
    keep, free = [G.State(wl.rowptr0, wl.col0, k=k, variant="rsvd", op="adj", precision=prec, L=L, P=P,
                          proj="lowrank") for _ in range(2)]
    for st in (keep, free):
        st.set_pairs(th0, X0)
    before = free.memory()
    free.release_graph()
    free.release_graph()  # a second call is a no-op
    m0 = int(wl.rowptr0[-1])
    assert free.memory() <= before - 2 * 4 * m0, (before, free.memory())
    assert free.shape()[1] == -1
    with pytest.raises(G.GrestError) as e:
        free.graph()
    assert e.value.status == G.EINVAL
    with pytest.raises(G.GrestError) as e:
        free.init_pairs(2)
    assert e.value.status == G.EINVAL
    d0 = wl.deltas[0]
    dev = torch.device("cuda:0")
    with pytest.raises(G.GrestError) as e:  # the first change listed twice, caught on the device
        free.update(0, torch.tensor(np.r_[d0.i[:3], d0.i[:1]], dtype=torch.int32, device=dev),
                    torch.tensor(np.r_[d0.j[:3], d0.j[:1]], dtype=torch.int32, device=dev),
                    torch.tensor(np.r_[d0.sign[:3], d0.sign[:1]], dtype=torch.int8, device=dev))
    assert e.value.status == G.EINVAL
    Xo, tho = X0, th0
    for t, d in enumerate(wl.deltas[:3]):
        om = W.omega(wl.cfg_id, 0, t + 1, d.n_new, L + P) if d.n_new > 0 else None
        for st in (keep, free):
            st.update_delta(d, om)
            st.sync()
        vk, Xk = keep.get()
        vf, Xf = free.get()
        assert np.array_equal(vk, vf) and np.array_equal(Xk, Xf), f"step {t + 1}: results differ"
        r = O.grest_step(A, Xo, tho, d.n_new, d.i, d.j, d.sign, k, variant="rsvd", op="adj", L=L, Omega=om,
                         proj="lowrank")
        check_step(free, r, "adj", prec, k, f"step {t + 1}")
        A, Xo, tho = r.A, r.X, r.theta
    keep.close()
    free.close()


@pytest.mark.parametrize("op,prec", [("adj", "fp64"), ("adj", "fp32"), ("lap", "mixed"), ("nlap", "fp64")])
def test_drift_matches_oracle_definition(op, prec):
    """The device's drift measure (orthonormality, scaled residual) against the oracle's
    definition evaluated on the same pairs and the oracle's graph, after three updates."""
    wl = W.preset("sbm_n2000", scale=0.5, steps=3)
    k = 8
    banner(f"drift op={op} prec={prec}")
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, shift0 = O.leading_eigenpairs(A, k, op)
    vals0 = th0 if op == "adj" else shift0 - th0
    st = G.State(wl.rowptr0, wl.col0, k=k, variant="g2", op=op, precision=prec)
    st.set_pairs(vals0, X0)
    for d in wl.deltas[:3]:
        st.update_delta(d)
        A = O.updated_adjacency(A, O.assemble_delta(A, d.n_new, d.i, d.j, d.sign))
    st.sync()
    vals, X = st.get()
    orth, resid = st.drift()
    o_ref, r_ref = O.drift_metrics(A, X, vals, op)
    banner(f"  orth {orth:.3e} (oracle {o_ref:.3e}), resid {resid:.3e} (oracle {r_ref:.3e})")
    assert abs(orth - o_ref) <= 1e-12, (orth, o_ref)
    assert abs(resid - r_ref) <= (1e-11 if prec == "fp64" else 1e-5), (resid, r_ref)
    st.close()


def test_restart_policy_recomputes_like_init_pairs():
    """With zero thresholds every check finds drift, so the pairs are recomputed right
    after the fifth update (min_gap = 5) and not at the sixth or seventh: the state then
    equals, bit for bit, a state without the policy that called grest_init_pairs with the
    same iterations and seed at that point.  Thresholds that are never reached leave the
    results bitwise those of a state without the policy."""
    wl = W.preset("sbm_n2000", scale=0.5, steps=7)
    k, iters, seed = 8, 40, 123
    banner("restart policy")
    mk = lambda: G.State(wl.rowptr0, wl.col0, k=k, variant="g2", op="adj", precision="fp64")
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, _ = O.leading_eigenpairs(A, k, "adj")
    pol, ref, lax = mk(), mk(), mk()
    for st in (pol, ref, lax):
        st.set_pairs(th0, X0)
    pol.set_restart(0.0, 0.0, check_every=1, min_gap=5, iterations=iters, seed=seed)
    lax.set_restart(1e30, 1e30, check_every=2, min_gap=0, iterations=iters, seed=seed)
    for t, d in enumerate(wl.deltas[:7]):
        for st in (pol, ref, lax):
            st.update_delta(d)
        if t == 4:
            ref.init_pairs(iters, seed)
        n_rs, lo, lr = pol.restart_stats()
        assert n_rs == (0 if t < 4 else 1), (t, n_rs)
        assert lo >= 0.0 and lr >= 0.0
    for st in (pol, ref, lax):
        st.sync()
    vp, Xp = pol.get()
    vr, Xr = ref.get()
    assert np.array_equal(vp, vr) and np.array_equal(Xp, Xr), "restart differs from init_pairs"
    assert lax.restart_stats()[0] == 0
    plain = mk()
    plain.set_pairs(th0, X0)
    for d in wl.deltas[:7]:
        plain.update_delta(d)
    plain.sync()
    vl, Xl = lax.get()
    v0, X0g = plain.get()
    assert np.array_equal(vl, v0) and np.array_equal(Xl, X0g), "the drift checks changed the results"
    for st in (pol, ref, lax, plain):
        st.close()


def test_restart_policy_argument_checks():
    banner("restart policy arguments")
    wl = W.preset("sbm_n2000", scale=0.25, steps=1)
    st = G.State(wl.rowptr0, wl.col0, k=4, variant="g2", op="adj", proj="lowrank")
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, _ = O.leading_eigenpairs(A, 4, "adj")
    st.set_pairs(th0, X0)
    for bad in [dict(check_every=-1), dict(min_gap=-1), dict(iterations=0)]:
        args = dict(tol_resid=1e-3, tol_orth=1e-3, check_every=1, min_gap=5, iterations=10)
        args.update(bad)
        with pytest.raises(G.GrestError) as e:
            st.set_restart(**args)
        assert e.value.status == G.EINVAL
    st.release_graph()
    with pytest.raises(G.GrestError) as e:  # a recomputation needs the graph
        st.set_restart(1e-3, 1e-3)
    assert e.value.status == G.EINVAL
    orth, resid = st.drift()
    assert orth <= 1e-12 and np.isnan(resid)
    st.close()


def test_lowrank_projection_limits():
    """The low-rank form is refused for the normalised Laplacian (its change rescales every
    row next to a node whose degree changed), and a Laplacian state keeps its graph."""
    banner("lowrank limits")
    wl = W.preset("sbm_n2000", scale=0.05, steps=1)
    with pytest.raises(G.GrestError) as e:
        G.State(wl.rowptr0, wl.col0, k=4, variant="g2", op="nlap", proj="lowrank")
    assert e.value.status == G.EINVAL
    st = G.State(wl.rowptr0, wl.col0, k=4, variant="g2", op="lap", proj="lowrank")
    with pytest.raises(G.GrestError) as e:
        st.release_graph()
    assert e.value.status == G.EINVAL
    st.close()
    st = G.State(wl.rowptr0, wl.col0, k=4, variant="g2", op="adj")
    with pytest.raises(G.GrestError) as e:  # the exact form needs its graph
        st.release_graph()
    assert e.value.status == G.EINVAL
    st.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_laplacian_k64_width_128(prec):
    """The large-graph form's shape at n0 = 2000: Chung-Lu (exponent 2.2) with 1 % node
    growth per step, combinatorial Laplacian, K = 64 smallest pairs, G-REST2, so the basis
    is 128 wide (the widest the kernels take: 128-column applies and products, the
    64-wide CholQR2 factor, the 128 template of the small eigensolver)."""
    wl = W.preset("chunglu_n4e6", scale=0.0005, steps=2)
    run_trajectory(wl, 64, "g2", "lap", prec, 2)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_laplacian_k65_rsvd_width_194(prec):
    """The large Laplacian workload's shape at n0 = 4000: Chung-Lu, combinatorial
    Laplacian, K = 65 (the 64 smallest non-trivial pairs and the trivial one), G-REST_RSVD
    with L = P = 64, so the basis is 194 wide (the small eigensolver's LDS-resident
    tridiagonalisation, the tall products and applies in blocks of 128 columns), 1 % node
    growth per step."""
    wl = W.preset("chunglu_n4e6", scale=0.001, steps=3)
    run_trajectory(wl, 65, "rsvd", "lap", prec, 3, L=64, P=64)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rsvd_sketch_rank_below_L(prec):
    """Fewer new nodes than L: the sketch keeps fewer than L columns, so the basis
    [X | R | Delta X] has dropped columns between its two packed blocks (the small
    eigensolver's index map)."""
    wl = W.sbm_small(n0=800, new_per_step=3, insertions=40, deletions=10, steps=3, cfg_id=1, graph_id=31)
    run_trajectory(wl, 8, "rsvd", "adj", prec, 3, L=8, P=8)


def test_rsvd_single_edge_without_new_nodes():
    """RSVD with no new node and one changed edge: R is empty and Delta X has rank <= 2."""
    banner("rsvd single edge flip")
    wl = W.preset("sbm_n2000", scale=0.05, steps=1)
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, _ = O.leading_eigenpairs(A, 4)
    st = G.State(wl.rowptr0, wl.col0, k=4, variant="rsvd", precision="fp64", L=4, P=4)
    st.set_pairs(th0, X0)
    Ad = A.toarray()
    i, j = map(int, np.argwhere(np.triu(Ad == 0, 1))[7])
    st.update(0, [i], [j], np.array([1], np.int8))
    st.sync()
    r = O.grest_step(A, X0, th0, 0, [i], [j], [1], 4, variant=O.RSVD, L=4)
    check_step(st, r, "adj", "fp64", 4, "rsvd single edge")
    st.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_kept_adjacency_product_matches_direct_product(prec):
    """For the adjacency the product A X of the tracked block is kept from the last
    back-projection and updated by Delta_1 X, so the sparse product only multiplies the new
    columns (with a full-width product every 16 updates).  Against a second state that is
    re-seeded with its own pairs before every update (which forces the full product) the
    trajectories agree to rounding over 20 updates, across the refresh."""
    wl = W.preset("sbm_n2000", scale=0.5, steps=20)
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, _ = O.leading_eigenpairs(A, 8, "adj")
    sa = G.State(wl.rowptr0, wl.col0, k=8, variant="rsvd", precision=prec, L=8, P=8)
    sb = G.State(wl.rowptr0, wl.col0, k=8, variant="rsvd", precision=prec, L=8, P=8)
    sa.set_pairs(th0, X0)
    sb.set_pairs(th0, X0)
    tol_v, tol_s = (1e-11, 1e-9) if prec == "fp64" else (1e-5, 1e-3)
    for t, d in enumerate(wl.deltas):
        banner(f"kept product step {t + 1} prec={prec}")
        om = W.omega(wl.cfg_id, 0, t + 1, d.n_new, 16) if d.n_new > 0 else None
        sa.update_delta(d, om)
        sa.sync()
        sb.update_delta(d, om)
        sb.sync()
        va, Xa = sa.get()
        vb, Xb = sb.get()
        kk = M.gap_prefix(np.abs(vb), 8, 1e-3)
        assert M.eig_rel_error(va, vb) <= tol_v, (t, M.eig_rel_error(va, vb))
        if kk > 0:
            assert M.subspace_sine(Xa[:, :kk], Xb[:, :kk]) <= tol_s
        sb.set_pairs(vb, Xb)  # drops the kept product: the next update multiplies all columns
    sa.close()
    sb.close()


# ------------------------------------------------------------------------------------
# edge cases
# ------------------------------------------------------------------------------------
def _small_state(prec="fp64", variant="g3", k=4, max_new=8):
    wl = W.preset("sbm_n2000", scale=0.05, steps=1)
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, _ = O.leading_eigenpairs(A, k)
    st = G.State(wl.rowptr0, wl.col0, k=k, variant=variant, precision=prec, max_new=max_new, L=4, P=4)
    st.set_pairs(th0, X0)
    return wl, A, th0, X0, st


def test_empty_update_keeps_pairs():
    banner("empty update")
    wl, A, th0, X0, st = _small_state()
    e = np.zeros(0, dtype=np.int64)
    st.update(0, e, e, e.astype(np.int8))
    st.sync()
    vals, X = st.get()
    assert M.eig_rel_error(vals, th0) < 1e-12
    assert M.subspace_sine(X, X0) < 1e-10


def test_isolated_new_nodes_keep_pairs():
    banner("isolated appended nodes")
    wl, A, th0, X0, st = _small_state()
    e = np.zeros(0, dtype=np.int64)
    st.update(3, e, e, e.astype(np.int8))
    st.sync()
    vals, X = st.get()
    assert X.shape[0] == A.shape[0] + 3
    assert M.eig_rel_error(vals, th0) < 1e-12
    assert np.abs(X[-3:]).max() == 0.0


def test_single_edge_update_rank_deficient_block():
    banner("single edge flip")
    wl, A, th0, X0, st = _small_state()
    Ad = A.toarray()
    i, j = map(int, np.argwhere(np.triu(Ad == 0, 1))[5])
    st.update(0, [i], [j], np.array([1], np.int8))
    st.sync()
    r = O.grest_step(A, X0, th0, 0, [i], [j], [1], 4, variant=O.G3)
    assert r.rank_W <= 2
    check_step(st, r, "adj", "fp64", 4, "single edge")


@pytest.mark.parametrize("bad", ["insert_existing", "delete_missing", "duplicate", "self_loop"])
def test_invalid_update_rejected_state_unchanged(bad):
    banner(f"invalid update: {bad}")
    wl, A, th0, X0, st = _small_state()
    rp0, col0 = st.graph()
    v0, Xs0 = st.get()
    Ad = A.toarray()
    ex = np.argwhere(np.triu(Ad == 1, 1))[0]
    mi = np.argwhere(np.triu(Ad == 0, 1))[0]
    cases = {
        "insert_existing": ([ex[0]], [ex[1]], [1]),
        "delete_missing": ([mi[0]], [mi[1]], [-1]),
        "duplicate": ([mi[0], mi[0]], [mi[1], mi[1]], [1, 1]),
        "self_loop": ([3], [3], [1]),
    }
    i, j, g = cases[bad]
    with pytest.raises(G.GrestError) as e:
        st.update(0, i, j, np.array(g, np.int8))
    assert e.value.status == G.EINVAL
    rp1, col1 = st.graph()
    v1, Xs1 = st.get()
    assert np.array_equal(rp0, rp1) and np.array_equal(col0, col1)
    assert np.array_equal(v0, v1) and np.array_equal(Xs0, Xs1)
    # the state still updates correctly afterwards
    d = wl.deltas[0]
    st.update_delta(d)
    st.sync()


def test_invalid_update_detected_on_device_for_device_inputs():
    """Membership errors in a change list that lives in device memory (no host check)."""
    import torch
    banner("device-side validation")
    wl, A, th0, X0, st = _small_state()
    Ad = A.toarray()
    ex = np.argwhere(np.triu(Ad == 1, 1))[0]
    dev = torch.device("cuda")
    i = torch.tensor([int(ex[0])], dtype=torch.int32, device=dev)
    j = torch.tensor([int(ex[1])], dtype=torch.int32, device=dev)
    g = torch.tensor([1], dtype=torch.int8, device=dev)
    with pytest.raises(G.GrestError) as e:
        st.update(0, i, j, g)
    assert e.value.status == G.EINVAL


def test_k_too_large_rejected():
    banner("k >= n")
    rp = np.array([0, 1, 2, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    with pytest.raises(G.GrestError):
        G.State(rp, col, k=3)


def test_deterministic_bitwise():
    banner("determinism")
    outs = []
    for _ in range(2):
        wl = W.preset("sbm_n1e6", scale=0.01, steps=2)
        A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
        th0, X0, _ = O.leading_eigenpairs(A, 8)
        st = G.State(wl.rowptr0, wl.col0, k=8, variant="rsvd", precision="fp32", L=8, P=8)
        st.set_pairs(th0, X0)
        for t, d in enumerate(wl.deltas):
            st.update_delta(d, W.omega(wl.cfg_id, 0, t + 1, d.n_new, 16))
        st.sync()
        outs.append(st.get(np.float32))
        st.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def _device_updates(wl, variant, L, P):
    import torch
    dev = torch.device("cuda")
    ups = []
    for t, d in enumerate(wl.deltas):
        om = None
        if variant == "rsvd" and d.n_new > 0:
            om = torch.tensor(W.omega(wl.cfg_id, 0, t + 1, d.n_new, L + P), dtype=torch.float64, device=dev)
        ups.append((d.n_new, torch.tensor(d.i, dtype=torch.int32, device=dev),
                    torch.tensor(d.j, dtype=torch.int32, device=dev),
                    torch.tensor(d.sign, dtype=torch.int8, device=dev), om))
    torch.cuda.synchronize()
    return ups


@pytest.mark.parametrize("case", ["sbm_adj_rsvd_fp32", "sbm_adj_rsvd_fp64", "chunglu_nlap_g2_fp64",
                                  "chunglu_lap_g3_mixed"])
def test_overlap_mode_matches_one_stream(case):
    """With the graph stage of each update on a second stream (grest_set_overlap), the
    updates give the same bits as on one stream: device-resident change lists queued back
    to back without a wait, the kept adjacency product, appended nodes, and a change list
    that the device rejects between two updates (the next update still waits for the
    rejected one's queued work)."""
    import torch
    wl_name, op, variant, prec = case.split("_")
    if wl_name == "sbm":
        wl = W.preset("sbm_n1e6", scale=0.01, steps=6)
    else:
        wl = W.preset("chunglu_n4e6", scale=0.002, steps=4)
    k, L, P = 8, 8, 8
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    th0, X0, shift0 = O.leading_eigenpairs(A, k, op)
    vals0 = th0 if op == "adj" else shift0 - th0
    ups = _device_updates(wl, variant, L, P)
    # an insertion of an edge that every graph of the run holds (the runs only insert
    # edges, or delete few): rejected on the device as an existing edge
    r0 = int(np.argmax(np.diff(wl.rowptr0) > 0))
    c0 = int(wl.col0[wl.rowptr0[r0]:wl.rowptr0[r0 + 1]].max())
    keep = all((d.sign > 0).all() for d in wl.deltas)
    dev = torch.device("cuda")
    bad = (torch.tensor([min(r0, c0)], dtype=torch.int32, device=dev),
           torch.tensor([max(r0, c0)], dtype=torch.int32, device=dev),
           torch.tensor([1], dtype=torch.int8, device=dev))
    outs = []
    for overlap in (False, True):
        banner(f"overlap={overlap} {case}")
        st = G.State(wl.rowptr0, wl.col0, k=k, variant=variant, op=op, precision=prec, L=L, P=P, max_new=96)
        st.set_pairs(vals0, X0)
        st.set_overlap(overlap)
        for t, (S, i, j, g, om) in enumerate(ups):
            st.update(S, i, j, g, om)
            if t == 1 and keep:
                with pytest.raises(G.GrestError) as e:
                    st.update(0, *bad)
                assert e.value.status == G.EINVAL
        st.sync()
        outs.append(st.get(np.float64) + st.graph())
        st.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("op,prec", [("adj", "fp64"), ("lap", "fp64"), ("nlap", "fp64"), ("adj", "fp32")])
def test_device_init_pairs_match_exact_leading_pairs(op, prec):
    """The device's initial eigensolver (Chebyshev-filtered block iteration with a residual
    stop) against dense eigh of the n = 2000 SBM's operator: it stops on its residual
    before the product budget, and every tracked pair is exact to the precision (FP64:
    eigenvalues to 1e-10, the separated subspace to 1e-8, the block orthonormal to 1e-12;
    FP32: 1e-5 and 1e-3)."""
    banner(f"device initial eigensolver op={op} prec={prec}")
    wl = W.preset("sbm_n2000", steps=0)
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    k = 8
    st = G.State(wl.rowptr0, wl.col0, k=k, variant="g3", op=op, precision=prec, max_new=100)
    tol = 1e-12 if prec == "fp64" else 4e-6
    products, resid = st.init_pairs(iterations=1500, seed=1, tol=tol)
    vals, X = st.get()
    th, Xe, shift = O.leading_eigenpairs(A, k + 1, op)
    ref = th if op == "adj" else shift - th
    if op == "adj":
        kk = M.gap_prefix(np.abs(th), k, 1e-3)
    else:
        kk = M.gap_prefix(ref, k, 1e-3, scale=float(np.abs(ref[:k]).max()))
    if op == "adj":
        e = M.eig_rel_error(vals, ref[:k])
    else:  # nu relative to the tracked spectrum's scale (nu_1 = 0 for L)
        e = float(np.abs(vals - ref[:k]).max() / np.abs(ref[:k]).max())
    sine = M.subspace_sine(X[:, :kk], Xe[:, :kk])
    orth = M.orthonormality(X)
    banner(f"  products {products}, resid {resid:.2e}, e_lambda {e:.2e}, sine(k*={kk}) {sine:.2e}, orth {orth:.2e}")
    assert products < 1500 and resid <= tol
    assert st.init_stats() == (products, resid)
    assert e <= TOL_EIG[prec], e
    assert sine <= TOL_SINE[prec], sine
    assert orth <= TOL_ORTH[prec], orth


def test_device_init_pairs_budget_and_arguments():
    """With a budget too small to converge the eigensolver keeps the last Rayleigh-Ritz
    pairs and reports their residual; bad arguments are refused."""
    banner("device initial eigensolver: budget and arguments")
    wl = W.preset("sbm_n2000", steps=0)
    st = G.State(wl.rowptr0, wl.col0, k=4, variant="g3", precision="fp64", max_new=8)
    products, resid = st.init_pairs(iterations=3, seed=2, tol=1e-14)
    assert products <= 3 and resid > 1e-14
    vals, X = st.get()
    assert np.all(np.isfinite(vals)) and M.orthonormality(X) <= 1e-12
    for bad in ((0, 1e-12), (10, -1.0), (10, float("nan"))):
        with pytest.raises(G.GrestError) as e:
            st.init_pairs(iterations=bad[0], seed=0, tol=bad[1])
        assert e.value.status == G.EINVAL


# ------------------------------------------------------------------------------------
# full size: the headline workload in the launch configuration the benchmark times
# ------------------------------------------------------------------------------------
def test_full_size_trajectory_parity():
    """n0 = 1e6 SBM, K = 32, RSVD with L = P = 32 (the benchmark's workload and kernel
    shapes): a 10-update trajectory from one shared start on the GPU (mixed and FP32) and
    in the oracle, compared after every update (eigenvalue error, subspace sine and
    orthonormality at the precision's tolerances).  The start is a few block power
    iterations on the host (no exact eigensolve at this size); parity is the agreement of
    the two trajectories on the same inputs."""
    steps = 10
    wl = W.preset("sbm_n1e6", scale=1.0, steps=steps)
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    X = W.random_orthonormal(wl.n0, 32, 5)
    for _ in range(6):  # block power iteration with Cholesky QR (host, FP64)
        Y = A @ X
        R = np.linalg.cholesky(Y.T @ Y).T
        X = np.linalg.solve(R.T, Y.T).T
    th = np.einsum("ij,ij->j", X, A @ X)
    oms = [W.omega(wl.cfg_id, 0, t + 1, d.n_new, 64) for t, d in enumerate(wl.deltas)]
    ref = []
    Ao, Xo, tho = A, X, th
    for t, d in enumerate(wl.deltas):
        banner(f"full size: oracle step {t + 1} n={Ao.shape[0]} nnz={Ao.nnz}")
        r = O.grest_step(Ao, Xo, tho, d.n_new, d.i, d.j, d.sign, 32, variant=O.RSVD, L=32, Omega=oms[t])
        ref.append(r)
        Ao, Xo, tho = r.A, r.X, r.theta
    n_fin = wl.n_at(steps) + 1
    nnz = int(wl.col0.size + 2 * sum(d.n_changes for d in wl.deltas) + 1024)
    for prec in ("mixed", "fp32"):
        st = G.State(wl.rowptr0, wl.col0, k=32, variant="rsvd", precision=prec, L=32, P=32, node_capacity=n_fin,
                     nnz_capacity=nnz)
        st.set_pairs(th, X)
        st.set_overlap(True)
        for t, d in enumerate(wl.deltas):
            banner(f"full size: GPU step {t + 1} prec={prec}")
            st.update_delta(d, oms[t])
            st.sync()
            check_step(st, ref[t], "adj", prec, 32, f"full size {prec} step {t + 1}")
        rp, col = st.graph()
        assert np.array_equal(rp, ref[-1].A.indptr) and np.array_equal(col, ref[-1].A.indices)
        st.close()
