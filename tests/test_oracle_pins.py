"""Pins of the FP64 oracle against facts that the paper and linear algebra fix.

None of these compares the oracle with itself: each checks it against a
worked example printed in the paper, a brute-force dense eigendecomposition, an
identity the paper proves, or a textbook invariant of the Rayleigh-Ritz
procedure.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import grest_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _graph(n, edges):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    i, j = e[:, 0], e[:, 1]
    return sp.csr_matrix((np.ones(2 * len(i)), (np.r_[i, j], np.r_[j, i])), shape=(n, n))


def fig1():
    g = json.load(open(os.path.join(GOLDEN, "fig1_update.json")))
    A = _graph(g["n_old"], [[a - 1, b - 1] for a, b in g["old_edges_1based"]])
    ch = np.asarray(g["changes_1based"])
    return g, A, ch[:, 0] - 1, ch[:, 1] - 1, ch[:, 2]


def random_case(seed, n=12, s=3, p=0.35, n_ins=4, n_del=3, connected=False):
    """A random small graph and a valid update (insertions, deletions, new nodes)."""
    rng = np.random.default_rng(seed)
    while True:
        U = np.triu(rng.random((n, n)) < p, 1)
        A = sp.csr_matrix((U | U.T).astype(float))
        if not connected:
            break
        from scipy.sparse.csgraph import connected_components
        if connected_components(A, directed=False)[0] == 1:
            break
    iu, ju = np.triu_indices(n, 1)
    present = U[iu, ju]
    ins = rng.choice(np.flatnonzero(~present), size=min(n_ins, (~present).sum()), replace=False)
    dele = rng.choice(np.flatnonzero(present), size=min(n_del, present.sum()), replace=False)
    if connected:  # keep old nodes attached: only delete edges whose endpoints keep degree >= 2
        deg = np.asarray(A.sum(1)).ravel()
        keep = []
        for q in dele:
            a, b = iu[q], ju[q]
            if deg[a] > 2 and deg[b] > 2:
                deg[a] -= 1
                deg[b] -= 1
                keep.append(q)
        dele = np.asarray(keep, dtype=np.int64)
    ei = list(iu[ins]) + list(iu[dele])
    ej = list(ju[ins]) + list(ju[dele])
    sg = [1] * len(ins) + [-1] * len(dele)
    for q in range(s):  # every new node gets >= 1 old partner, plus random new-new edges
        v = n + q
        partners = rng.choice(n, size=rng.integers(1, 4), replace=False)
        for a in partners:
            ei.append(int(a)); ej.append(v); sg.append(1)
        for w in range(n, v):
            if rng.random() < 0.4:
                ei.append(w); ej.append(v); sg.append(1)
    return A, np.asarray(ei), np.asarray(ej), np.asarray(sg)


# ------------------------------------------------------------------------------------
# worked example (Fig. 1)
# ------------------------------------------------------------------------------------
def test_fig1_delta_blocks_match_caption():
    g, A, ei, ej, sg = fig1()
    D = O.assemble_delta(A, g["n_new"], ei, ej, sg).toarray()
    n = g["n_old"]
    K = np.zeros((n, n))
    for a, b, v in g["caption_K_1based"]:
        K[a - 1, b - 1] = v
    G = np.zeros((n, g["n_new"]))
    for a, b, v in g["caption_G_1based"]:
        G[a - 1, b - 1] = v
    assert np.array_equal(D[:n, :n], K)
    assert np.array_equal(D[:n, n:], G)
    assert np.array_equal(D[n:, :n], G.T)
    assert np.count_nonzero(D[n:, n:]) == g["caption_C_nonzeros"]


def test_fig1_full_rank_subspace_is_exact():
    """K=3: the G-REST3 subspace spans all of R^8, so Ritz pairs = eigenpairs of A^(t+1)."""
    g, A, ei, ej, sg = fig1()
    th0, X0, _ = O.leading_eigenpairs(A, 3)
    r = O.grest_step(A, X0, th0, g["n_new"], ei, ej, sg, 3, variant=O.G3)
    assert r.Z.shape[1] == 8
    ev, EV = np.linalg.eigh(r.A.toarray())
    order = O.select(ev, 3, "LM")
    assert np.allclose(r.theta, ev[order], atol=1e-12, rtol=0)
    for c in range(3):
        assert abs(abs(r.X[:, c] @ EV[:, order[c]]) - 1) < 1e-12


def test_fig1_g2_misses_new_node_information():
    """G-REST2 (no Delta_2 block) spans a smaller subspace and cannot be exact here."""
    g, A, ei, ej, sg = fig1()
    th0, X0, _ = O.leading_eigenpairs(A, 3)
    r2 = O.grest_step(A, X0, th0, g["n_new"], ei, ej, sg, 3, variant=O.G2)
    ev = np.linalg.eigvalsh(r2.A.toarray())
    assert r2.Z.shape[1] < 8
    assert np.max(np.abs(r2.theta - ev[O.select(ev, 3, "LM")])) > 1e-3


# ------------------------------------------------------------------------------------
# brute force: whenever the subspace is all of R^n', the update is exact
# ------------------------------------------------------------------------------------
@pytest.mark.parametrize("op", [O.ADJ, O.LAP, O.NLAP])
@pytest.mark.parametrize("seed", range(6))
def test_full_rank_subspace_reproduces_dense_eigh(op, seed):
    A, ei, ej, sg = random_case(seed, n=8, s=3, p=0.45, connected=(op != O.ADJ))
    k = 6
    th0, X0, _ = O.leading_eigenpairs(A, k, op)
    r = O.grest_step(A, X0, th0, 3, ei, ej, sg, k, variant=O.G3, op=op)
    n2 = A.shape[0] + 3
    if r.Z.shape[1] < n2:
        pytest.skip("subspace not full rank for this draw")
    T, _ = O.operator_matrix(r.A, op)
    ev, EV = np.linalg.eigh(T.toarray())
    order = O.select(ev, k, O.which_for(op))
    assert np.allclose(r.theta, ev[order], atol=1e-11 * max(1, abs(ev).max()), rtol=0)


def test_full_rank_occurs_in_brute_force_cases():
    hits = 0
    for seed in range(6):
        A, ei, ej, sg = random_case(seed, n=8, s=3, p=0.45)
        th0, X0, _ = O.leading_eigenpairs(A, 6)
        r = O.grest_step(A, X0, th0, 3, ei, ej, sg, 6, variant=O.G3)
        hits += r.Z.shape[1] == 11
    assert hits >= 3


# ------------------------------------------------------------------------------------
# identities proved in the paper
# ------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_prop3_delta_xbar_equals_delta1_x(seed):
    A, ei, ej, sg = random_case(seed, n=30, s=5)
    n = A.shape[0]
    D = O.assemble_delta(A, 5, ei, ej, sg)
    X = np.random.default_rng(seed).standard_normal((n, 4))
    lhs = D @ O.pad_rows(X, 5)
    rhs = D[:, :n] @ X
    assert np.array_equal(lhs, rhs)


@pytest.mark.parametrize("seed", range(6))
def test_prop4_rank_of_delta2(seed):
    rng = np.random.default_rng(seed)
    n, s = 40, 9
    A = sp.csr_matrix((n, n))
    # sparse wiring: few old partners (J) and few connected new nodes (Q)
    J = rng.choice(n, size=rng.integers(1, 6), replace=False)
    Qn = rng.choice(s, size=rng.integers(1, 7), replace=False)
    ei, ej = [], []
    for q in Qn:
        for a in rng.choice(J, size=rng.integers(1, len(J) + 1), replace=False):
            ei.append(int(a)); ej.append(n + int(q))
    D = O.assemble_delta(A, s, ei, ej, np.ones(len(ei))).toarray()
    D2 = D[:, n:]
    JJ = np.count_nonzero(np.abs(D2[:n]).sum(1))
    QQ = np.count_nonzero(np.abs(D2[:n]).sum(0))
    assert np.linalg.matrix_rank(D2) <= min(JJ, QQ)


@pytest.mark.parametrize("seed", range(5))
def test_rsvd_is_exact_when_rank_below_sketch(seed):
    """Sec. 3.5: rank((I-Pi) Delta_2) < L+P  =>  RSVD returns its range; with rank <= L the
    G-REST_RSVD Ritz pairs equal the G-REST3 ones."""
    A, ei, ej, sg = random_case(seed, n=40, s=4, p=0.15)
    k, L, P = 4, 6, 4
    th0, X0, _ = O.leading_eigenpairs(A, k)
    Om = np.random.default_rng(100 + seed).standard_normal((4, L + P))
    r3 = O.grest_step(A, X0, th0, 4, ei, ej, sg, k, variant=O.G3)
    rr = O.grest_step(A, X0, th0, 4, ei, ej, sg, k, variant=O.RSVD, L=L, Omega=Om)
    assert np.allclose(rr.theta, r3.theta, atol=1e-12, rtol=0)
    sub = np.linalg.svd(r3.X.T @ rr.X, compute_uv=False)
    assert np.all(sub > 1 - 1e-12)


def test_rsvd_truncates_when_rank_exceeds_L():
    A, ei, ej, sg = random_case(7, n=60, s=12, p=0.1)
    k, L, P = 4, 3, 3
    th0, X0, _ = O.leading_eigenpairs(A, k)
    Om = np.random.default_rng(1).standard_normal((12, L + P))
    rr = O.grest_step(A, X0, th0, 12, ei, ej, sg, k, variant=O.RSVD, L=L, Omega=Om)
    r3 = O.grest_step(A, X0, th0, 12, ei, ej, sg, k, variant=O.G3)
    assert rr.Z.shape[1] <= 2 * k + L < r3.Z.shape[1]


def _rsvd_truncation_case(seed):
    """An update whose projected trailing block has rank r with L < r < L + P, and the
    dense leading-L left singular subspace of that block computed directly."""
    A, ei, ej, sg = random_case(seed, n=80, s=8, p=0.08, n_ins=6, n_del=4)
    k, L, P, s = 4, 3, 8, 8
    n = A.shape[0]
    _, X0, _ = O.leading_eigenpairs(A, k)
    Xb = np.vstack([X0, np.zeros((s, k))])
    # Delta_2 straight from the change list: the appended nodes' columns of Delta
    D2 = np.zeros((n + s, s))
    for a, b, g in zip(ei, ej, sg):
        if b >= n:
            D2[a, b - n] += g
            if a >= n:
                D2[b, a - n] += g
    P_perp = np.eye(n + s) - Xb @ Xb.T
    # SciPy's SVD (not NumPy's, which the planted-mistake tests replace inside the oracle)
    U, sig, _ = sla.svd(P_perp @ D2, full_matrices=False)
    r = int(np.count_nonzero(sig > 1e-10 * sig[0]))
    Om = np.random.default_rng(500 + seed).standard_normal((s, L + P))
    return A, Xb, ei, ej, sg, n, s, L, P, U[:, :L], sig, r, Om


def _rsvd_truncation_sine(seed):
    A, Xb, ei, ej, sg, n, s, L, P, UL, sig, r, Om = _rsvd_truncation_case(seed)
    D = O.assemble_delta(A, s, ei, ej, sg)
    _, DT, _, _ = O.operator_delta(A, O.updated_adjacency(A, D), O.ADJ)
    R = O.rsvd_basis(Xb, DT[:, n:].tocsr(), Om, L)
    if R.shape[1] != L:
        return np.inf
    # sine of the largest principal angle = ||U_L U_L^T - R R^T||_2 for orthonormal blocks
    return float(np.linalg.norm(UL @ UL.T - R @ R.T, 2))


@pytest.mark.parametrize("seed", range(6))
def test_rsvd_truncation_keeps_leading_left_singular_subspace(seed):
    """Sec. 3.5, S.2-S.4: when L < rank((I - Pi) Delta_2) < L + P the Gaussian sketch spans
    the whole range (probability 1), so M U_L is exactly the span of the L leading left
    singular vectors of the dense (I - Pi) Delta_2."""
    _, _, _, _, _, _, _, L, P, _, sig, r, _ = _rsvd_truncation_case(seed)
    assert L < r < L + P
    assert (sig[L - 1] - sig[L]) / sig[0] > 0.02  # a gap that makes the subspace well defined
    assert _rsvd_truncation_sine(seed) < 1e-12


def test_planted_trailing_singular_vectors_are_caught(monkeypatch):
    real = np.linalg.svd

    def trailing_first(a, full_matrices=True, compute_uv=True, **kw):
        U, s, Vt = real(a, full_matrices=full_matrices, compute_uv=True, **kw)
        return U[:, ::-1], s[::-1], Vt[::-1]
    assert _rsvd_truncation_sine(1) < 1e-12
    monkeypatch.setattr(O.np.linalg, "svd", trailing_first)
    assert _rsvd_truncation_sine(1) > 1e-3


def test_planted_right_for_left_singular_vectors_is_caught(monkeypatch):
    real = np.linalg.svd

    def right_for_left(a, full_matrices=True, compute_uv=True, **kw):
        U, s, Vt = real(a, full_matrices=full_matrices, compute_uv=True, **kw)
        return Vt.T[: U.shape[0], : U.shape[1]], s, Vt
    monkeypatch.setattr(O.np.linalg, "svd", right_for_left)
    assert _rsvd_truncation_sine(1) > 1e-3


# ------------------------------------------------------------------------------------
# Rayleigh-Ritz invariants (Alg. 1, Galerkin condition, Thm. 1, interlacing)
# ------------------------------------------------------------------------------------
@pytest.mark.parametrize("variant", [O.G2, O.G3])
@pytest.mark.parametrize("op", [O.ADJ, O.LAP, O.NLAP])
def test_ritz_invariants(variant, op):
    A, ei, ej, sg = random_case(3, n=60, s=6, p=0.12, n_ins=10, n_del=6, connected=True)
    k = 5
    th0, X0, _ = O.leading_eigenpairs(A, k, op)
    r = O.grest_step(A, X0, th0, 6, ei, ej, sg, k, variant=variant, op=op)
    T, _ = O.operator_matrix(r.A, op)
    T = T.toarray()
    Z = r.Z
    nrm = np.abs(np.linalg.eigvalsh(T)).max()
    # orthonormal basis and orthonormal Ritz vectors
    assert np.abs(Z.T @ Z - np.eye(Z.shape[1])).max() < 1e-13
    assert np.abs(r.X.T @ r.X - np.eye(k)).max() < 1e-13
    # Galerkin: Z^T (T x - theta x) = 0
    R = T @ r.X - r.X * r.theta
    assert np.abs(Z.T @ R).max() < 1e-12 * nrm
    # Thm. 1: ||T Z - Z H||_2 = ||Z_perp^T T Z||_2
    Qf, _ = np.linalg.qr(np.hstack([Z, np.random.default_rng(0).standard_normal((Z.shape[0], Z.shape[0]))]))
    Zp = Qf[:, Z.shape[1]:]
    lhs = np.linalg.norm(T @ Z - Z @ r.H, 2)
    rhs = np.linalg.norm(Zp.T @ T @ Z, 2)
    assert abs(lhs - rhs) < 1e-11 * nrm
    # Cauchy interlacing: j-th largest Ritz value <= j-th largest eigenvalue, and mirrored
    ev = np.sort(np.linalg.eigvalsh(T))
    rv = np.sort(np.linalg.eigvalsh(r.H))
    d = rv.size
    assert np.all(rv[::-1] <= ev[::-1][:d] + 1e-11 * nrm)
    assert np.all(rv >= ev[:d] - 1e-11 * nrm)


def test_g3_dominates_g2_by_courant_fischer():
    """span(G-REST2) is inside span(G-REST3), so every top-j algebraic Ritz value of G3 is >=
    that of G2 (and every bottom-j one is <=)."""
    for seed in range(4):
        A, ei, ej, sg = random_case(seed, n=50, s=8, p=0.15, n_ins=8, n_del=5)
        th0, X0, _ = O.leading_eigenpairs(A, 4)
        r2 = O.grest_step(A, X0, th0, 8, ei, ej, sg, 4, variant=O.G2)
        r3 = O.grest_step(A, X0, th0, 8, ei, ej, sg, 4, variant=O.G3)
        a2 = np.sort(np.linalg.eigvalsh(r2.H))[::-1]
        a3 = np.sort(np.linalg.eigvalsh(r3.H))[::-1]
        assert np.all(a3[:a2.size] >= a2 - 1e-11)
        assert np.all(a3[::-1][:a2.size] <= a2[::-1] + 1e-11)


# ------------------------------------------------------------------------------------
# special cases
# ------------------------------------------------------------------------------------
@pytest.mark.parametrize("op", [O.ADJ, O.LAP, O.NLAP])
def test_empty_update_returns_previous_pairs(op):
    A, _, _, _ = random_case(11, n=40, p=0.2, connected=True)
    k = 5
    th0, X0, _ = O.leading_eigenpairs(A, k, op)
    e = np.zeros(0, dtype=np.int64)
    for proj in (O.EXACT, O.LOWRANK):
        r = O.grest_step(A, X0, th0, 0, e, e, e, k, variant=O.G3, op=op, proj=proj)
        assert r.rank_W == 0
        assert np.allclose(r.theta, th0, atol=1e-12 * max(1, abs(th0).max()), rtol=0)
        assert np.all(np.linalg.svd(r.X.T @ X0, compute_uv=False) > 1 - 1e-12)


def test_lowrank_empty_update_is_exactly_identity_on_pairs():
    A, _, _, _ = random_case(12, n=30, p=0.2)
    X0 = np.linalg.qr(np.random.default_rng(0).standard_normal((30, 4)))[0]
    th0 = np.array([5.0, -3.0, 2.0, 1.0])
    e = np.zeros(0, dtype=np.int64)
    r = O.grest_step(A, X0, th0, 0, e, e, e, 4, variant=O.G3, proj=O.LOWRANK)
    assert np.allclose(r.theta, th0, atol=1e-13, rtol=0)


def test_laplacian_shift_identity_and_nonnegativity():
    A, ei, ej, sg = random_case(5, n=60, s=6, p=0.12, connected=True)
    k = 6
    th0, X0, _ = O.leading_eigenpairs(A, k, O.LAP)
    r = O.grest_step(A, X0, th0, 6, ei, ej, sg, k, variant=O.G3, op=O.LAP)
    d = np.asarray(r.A.sum(1)).ravel()
    assert r.shift == 2 * d.max()
    Lm = (sp.diags(d) - r.A).toarray()
    nu_rayleigh = np.einsum("ij,ij->j", r.X, Lm @ r.X)
    assert np.allclose(r.nu, nu_rayleigh, atol=1e-10)
    assert np.all(r.nu >= -1e-12)


def test_laplacian_null_vector_is_kept_on_connected_graph():
    """With G-REST3 and the exact projection, 1/sqrt(n') stays in the subspace even when alpha
    changes, so the smallest nu is 0 with the constant eigenvector."""
    A, ei, ej, sg = random_case(8, n=60, s=6, p=0.12, connected=True)
    k = 5
    th0, X0, _ = O.leading_eigenpairs(A, k, O.LAP)
    r = O.grest_step(A, X0, th0, 6, ei, ej, sg, k, variant=O.G3, op=O.LAP)
    from scipy.sparse.csgraph import connected_components
    assert connected_components(r.A, directed=False)[0] == 1
    one = np.ones(r.A.shape[0]) / np.sqrt(r.A.shape[0])
    assert abs(r.nu[0]) < 1e-10
    assert abs(abs(r.X[:, 0] @ one) - 1) < 1e-10


def test_normalized_laplacian_range():
    A, ei, ej, sg = random_case(9, n=60, s=6, p=0.12, connected=True)
    th0, X0, _ = O.leading_eigenpairs(A, 6, O.NLAP)
    r = O.grest_step(A, X0, th0, 6, ei, ej, sg, 6, variant=O.G3, op=O.NLAP)
    assert np.all(r.nu >= -1e-12) and np.all(r.nu <= 2 + 1e-12)
    # connected graph: nu_1 = 0 with eigenvector D^{1/2} 1 (normalised)
    d = np.asarray(r.A.sum(1)).ravel()
    v = np.sqrt(d) / np.linalg.norm(np.sqrt(d))
    ev = np.linalg.eigvalsh(np.eye(d.size) - np.diag(d ** -0.5) @ r.A.toarray() @ np.diag(d ** -0.5))
    assert abs(ev[0]) < 1e-10
    assert r.nu[0] >= -1e-12


@pytest.mark.parametrize("bad", ["insert_existing", "delete_missing", "self_loop", "dup",
                                 "out_of_range", "delete_new"])
def test_invalid_updates_are_rejected(bad):
    A = _graph(4, [[0, 1], [1, 2]])
    cases = {
        "insert_existing": ([0], [1], [1], 0),
        "delete_missing": ([0], [3], [-1], 0),
        "self_loop": ([2], [2], [1], 0),
        "dup": ([0, 0], [2, 2], [1, 1], 0),
        "out_of_range": ([0], [9], [1], 1),
        "delete_new": ([0], [4], [-1], 1),
    }
    ei, ej, sg, s = cases[bad]
    with pytest.raises(O.DeltaError):
        O.assemble_delta(A, s, ei, ej, sg)


def test_selection_order_and_ties():
    th = np.array([-3.0, -1.0, 1.0, 3.0, 0.5])
    assert list(O.select(th, 4, "LM")) == [3, 0, 2, 1]
    assert list(O.select(th, 3, "LA")) == [3, 2, 4]


# ------------------------------------------------------------------------------------
# the pins are sensitive: plant a mistake in the oracle and one of them fails
# ------------------------------------------------------------------------------------
def _fig1_truth():
    """Eigenvalues of the updated Fig. 1 graph, built directly from its edge lists."""
    g = json.load(open(os.path.join(GOLDEN, "fig1_update.json")))
    edges = {tuple(sorted((a - 1, b - 1))) for a, b in g["old_edges_1based"]}
    for a, b, v in g["changes_1based"]:
        e = tuple(sorted((a - 1, b - 1)))
        if v > 0:
            edges.add(e)
        else:
            edges.discard(e)
    M = np.zeros((8, 8))
    for a, b in edges:
        M[a, b] = M[b, a] = 1.0
    return np.linalg.eigvalsh(M)


def _full_rank_pin_holds():
    g, A, ei, ej, sg = fig1()
    th0, X0, _ = O.leading_eigenpairs(A, 3)
    r = O.grest_step(A, X0, th0, g["n_new"], ei, ej, sg, 3, variant=O.G3)
    ev = _fig1_truth()
    order = np.lexsort((np.arange(8), -ev, -np.abs(ev)))[:3]
    return np.allclose(r.theta, ev[order], atol=1e-10)


def test_unplanted_pin_holds():
    assert _full_rank_pin_holds()


def test_planted_sign_flip_in_delta_is_caught(monkeypatch):
    real = O.assemble_delta

    def flipped(A, s, i, j, g):
        D = real(A, s, i, j, g).tocsr(copy=True)
        D.data = np.where(D.data < 0, 1.0, D.data)  # a deletion mistaken for an insertion
        return D
    monkeypatch.setattr(O, "assemble_delta", flipped)
    assert not _full_rank_pin_holds()


def test_planted_wrong_selection_is_caught(monkeypatch):
    real = O.select
    monkeypatch.setattr(O, "select", lambda th, k, which: real(th, k, "LA"))
    assert not _full_rank_pin_holds()


def _isolated_nodes_pin_holds():
    """Appending isolated nodes leaves the spectrum and the padded eigenvectors unchanged."""
    A, _, _, _ = random_case(4, n=30, p=0.2)
    th0, X0, _ = O.leading_eigenpairs(A, 4)
    e = np.zeros(0, dtype=np.int64)
    r = O.grest_step(A, X0, th0, 3, e, e, e, 4, variant=O.G3)
    Xb = np.vstack([X0, np.zeros((3, 4))])
    return (np.allclose(r.theta, th0, atol=1e-12)
            and np.all(np.linalg.svd(r.X.T @ Xb, compute_uv=False) > 1 - 1e-12))


def test_isolated_new_nodes_keep_the_pairs():
    assert _isolated_nodes_pin_holds()


def test_planted_padding_at_top_is_caught(monkeypatch):
    monkeypatch.setattr(O, "pad_rows", lambda X, s: np.vstack([np.zeros((s, X.shape[1])), X]))
    assert not _isolated_nodes_pin_holds()


def test_planted_dropped_delta2_is_caught(monkeypatch):
    real = O.grest_step

    def g3_as_g2(*a, **kw):
        kw["variant"] = O.G2
        return real(*a, **kw)
    monkeypatch.setattr(O, "grest_step", g3_as_g2)
    assert not _full_rank_pin_holds()


def test_planted_missing_projection_is_caught(monkeypatch):
    monkeypatch.setattr(O, "project_out", lambda Xbar, W, passes=2: W)
    A, ei, ej, sg = random_case(3, n=40, s=4, p=0.15)
    th0, X0, _ = O.leading_eigenpairs(A, 4)
    r = O.grest_step(A, X0, th0, 4, ei, ej, sg, 4, variant=O.G3)
    assert np.abs(r.Z.T @ r.Z - np.eye(r.Z.shape[1])).max() > 1e-6


def test_planted_lowrank_without_delta_term_is_caught(monkeypatch):
    """Dropping Z^T Delta Z from the truncated projection breaks the full-rank pin."""
    real = O.operator_delta

    def no_delta(A_old, A_new, op):
        T_new, DT, c0, c1 = real(A_old, A_new, op)
        return T_new, DT * 0.0, c0, c1
    g, A, ei, ej, sg = fig1()
    th0, X0, _ = O.leading_eigenpairs(A, 3)
    ok = O.grest_step(A, X0, th0, 2, ei, ej, sg, 3, variant=O.G3, proj=O.LOWRANK)
    monkeypatch.setattr(O, "operator_delta", no_delta)
    bad = O.grest_step(A, X0, th0, 2, ei, ej, sg, 3, variant=O.G3, proj=O.LOWRANK)
    assert not np.allclose(ok.theta, bad.theta, atol=1e-6)


@pytest.mark.parametrize("op", [O.LAP, O.NLAP])
def test_laplacian_quadratic_form_matches_dense_definition(op):
    A, ei, ej, sg = random_case(13, n=50, s=5, p=0.1)
    A = O.updated_adjacency(A, O.assemble_delta(A, 5, ei, ej, sg))  # may contain isolated nodes
    X = np.random.default_rng(2).standard_normal((A.shape[0], 3))
    d = np.asarray(A.sum(1)).ravel()
    if op == O.LAP:
        Lm = np.diag(d) - A.toarray()
    else:
        s = np.where(d > 0, 1 / np.sqrt(np.maximum(d, 1e-300)), 0.0)
        Lm = np.eye(d.size) - np.diag(s) @ A.toarray() @ np.diag(s)
    ref = np.einsum("ij,ij->j", X, Lm @ X)
    assert np.allclose(O.laplacian_quadratic_form(A, X, op), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("op", [O.LAP, O.NLAP])
def test_ritz_nu_identity(op):
    """For Ritz vectors of T = shift I - L, the quadratic form equals shift - theta (Sec. 4.2)."""
    A, ei, ej, sg = random_case(5, n=60, s=6, p=0.12, connected=True)
    th0, X0, _ = O.leading_eigenpairs(A, 6, op)
    r = O.grest_step(A, X0, th0, 6, ei, ej, sg, 6, variant=O.G3, op=op)
    assert np.allclose(r.nu_rq, r.nu, atol=1e-11 * max(1.0, r.shift))


# ------------------------------------------------------------------------------------
# drift of tracked pairs (the restart measure): pinned by exact pairs from a dense
# eigensolver of matrices built here, and by closed forms of a scaled and a rotated pair
# ------------------------------------------------------------------------------------
def _small_graph(seed, n=60, p=0.12):
    rng = np.random.default_rng(seed)
    U = np.triu((rng.random((n, n)) < p).astype(np.float64), 1)
    Ad = U + U.T
    return Ad, sp.csr_matrix(Ad)


def _dense_reported_matrix(Ad, op):
    """A, L = D - A or L_n = I - D^-1/2 A D^-1/2 (identity rows for isolated nodes), built
    directly from their definitions."""
    d = Ad.sum(axis=1)
    if op == "adj":
        return Ad
    if op == "lap":
        return np.diag(d) - Ad
    s = np.where(d > 0, 1.0 / np.sqrt(np.where(d > 0, d, 1.0)), 0.0)
    return np.eye(len(d)) - s[:, None] * Ad * s[None, :]


@pytest.mark.parametrize("op", ["adj", "lap", "nlap"])
def test_drift_is_zero_on_exact_pairs(op):
    Ad, A = _small_graph(11)
    w, V = np.linalg.eigh(_dense_reported_matrix(Ad, op))
    idx = np.argsort(-np.abs(w))[:6] if op == "adj" else np.arange(6)
    orth, resid = O.drift_metrics(A, V[:, idx], w[idx], op)
    assert orth <= 1e-13 and resid <= 1e-13, (orth, resid)


def test_drift_of_scaled_pairs_is_orthonormality_only():
    Ad, A = _small_graph(12)
    w, V = np.linalg.eigh(Ad)
    idx = np.argsort(-np.abs(w))[:5]
    eps = 1e-3
    orth, resid = O.drift_metrics(A, (1 + eps) * V[:, idx], w[idx], "adj")
    assert abs(orth - (2 * eps + eps * eps)) <= 1e-12, orth
    assert resid <= 1e-13, resid


@pytest.mark.parametrize("op", ["adj", "lap"])
def test_drift_of_rotated_pair_is_sine_times_gap(op):
    """x_1 = cos(phi) u_a + sin(phi) u_b reported with value lambda_a: its residual is
    |sin(phi)| |lambda_b - lambda_a|, divided by the scale (max |values| for the
    adjacency, 2 d_max for the Laplacian); orthonormality is untouched."""
    Ad, A = _small_graph(13)
    w, V = np.linalg.eigh(_dense_reported_matrix(Ad, op))
    order = np.argsort(-np.abs(w)) if op == "adj" else np.arange(len(w))
    keep, b = order[:4], order[10]
    phi = 0.2
    X = V[:, keep].copy()
    X[:, 0] = np.cos(phi) * V[:, keep[0]] + np.sin(phi) * V[:, b]
    orth, resid = O.drift_metrics(A, X, w[keep], op)
    scale = np.abs(w[keep]).max() if op == "adj" else 2.0 * Ad.sum(axis=1).max()
    expect = abs(np.sin(phi)) * abs(w[b] - w[keep[0]]) / scale
    assert orth <= 1e-13, orth
    assert abs(resid - expect) <= 1e-12 * max(1.0, expect), (resid, expect)


# ------------------------------------------------------------------------------------
# the truncated form (eq. RR_eigen_graph_upd_main3) against the exact one: when the old
# adjacency has rank K and its K nonzero pairs are tracked exactly, A = Xbar Theta Xbar^T,
# so both forms project the same matrix and must agree for any update
# ------------------------------------------------------------------------------------
@pytest.mark.parametrize("variant", ["g2", "g3", "rsvd"])
def test_lowrank_equals_exact_on_a_rank_k_graph(variant):
    a, b = 5, 7  # complete bipartite K_{5,7}: rank 2, eigenvalues +-sqrt(35), the rest 0
    n = a + b
    Ad = np.zeros((n, n))
    Ad[:a, a:] = 1.0
    Ad[a:, :a] = 1.0
    A = sp.csr_matrix(Ad)
    w, V = np.linalg.eigh(Ad)
    idx = np.argsort(-np.abs(w))[:2]
    th0, X0 = w[idx], V[:, idx]
    assert np.allclose(np.abs(th0), np.sqrt(a * b), atol=1e-12)
    # an update: two appended nodes, one insertion inside a side, one deletion across
    s_new = 2
    ei = np.array([0, 1, 3, 6, 2], dtype=np.int64)
    ej = np.array([1, 12, 13, 13, 9], dtype=np.int64)
    sg = np.array([1, 1, 1, 1, -1], dtype=np.int8)
    L = 2 if variant == "rsvd" else None
    om = np.random.default_rng(3).standard_normal((s_new, 4)) if variant == "rsvd" else None
    kw = dict(variant=variant, L=L, Omega=om)
    ex = O.grest_step(A, X0, th0, s_new, ei, ej, sg, 2, proj=O.EXACT, **kw)
    lr = O.grest_step(A, X0, th0, s_new, ei, ej, sg, 2, proj=O.LOWRANK, **kw)
    assert np.allclose(lr.theta, ex.theta, atol=1e-12, rtol=0), (lr.theta, ex.theta)
    # same Ritz subspace (signs aside)
    assert np.abs(np.abs(np.diag(lr.X.T @ ex.X)) - 1.0).max() <= 1e-10


# the truncated form for the shifted Laplacians (Sec. 4.2 with eq. RR_eigen_graph_upd_main3):
# when Xbar holds every pair of the old operator T, pad(T) = Xbar Theta Xbar^T exactly, so
# the truncated and the exact projected matrices coincide for any update
@pytest.mark.parametrize("op", ["lap", "nlap"])
def test_lowrank_equals_exact_for_laplacians_with_all_pairs(op):
    rng = np.random.default_rng(11)
    n = 14
    up = np.triu(rng.random((n, n)) < 0.3, 1)
    A = sp.csr_matrix((up | up.T).astype(float))
    th0, X0, _ = O.leading_eigenpairs(A, n, op)
    assert X0.shape == (n, n)
    s_new = 2
    ei = np.array([0, 2, 5, 1, 7], dtype=np.int64)
    ej = np.array([14, 15, 15, 3, 9], dtype=np.int64)
    Ad = A.toarray()
    sg = np.array([1, 1, 1, -1 if Ad[1, 3] else 1, -1 if Ad[7, 9] else 1], dtype=np.int8)
    ex = O.grest_step(A, X0, th0, s_new, ei, ej, sg, n, variant=O.G2, op=op, proj=O.EXACT)
    lr = O.grest_step(A, X0, th0, s_new, ei, ej, sg, n, variant=O.G2, op=op, proj=O.LOWRANK)
    assert np.allclose(lr.theta, ex.theta, atol=1e-10, rtol=0), (lr.theta, ex.theta)
