"""FP64 CPU oracle of the G-REST eigenpair update.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The GPU library never calls it and
shares no code with it.

What it computes (Eini, Karaaslanli, Kalantzis, Traganitis, "Subspace
Projection Methods for Fast Spectral Embeddings of Evolving Graphs"):

* the graph transition model of Sec. 2 (eq. adj_update): the padded old
  matrix plus a symmetric update Delta = [[K, G], [G^T, C]];
* the Rayleigh-Ritz procedure of Alg. 1 over the subspaces of Table 1:
  G-REST2 (previous eigenvectors plus the projected residual directions),
  G-REST3 (adds the projected trailing block Delta_2, Sec. 3.3) and
  G-REST_RSVD (replaces Delta_2 by the rank-L randomized basis of Sec. 3.5,
  steps S.1-S.4);
* the tracking step of Alg. 2 with either the projection onto the updated
  matrix (eq. RR_eigen_graph_upd_main2, "exact") or the truncated form that
  replaces the old matrix by its rank-K eigendecomposition
  (eq. RR_eigen_graph_upd_main3, "lowrank");
* the shifted Laplacians of Sec. 4.2: T = alpha I - L with alpha = 2 d_max, and
  T_n = 2 I - L_n; their leading pairs are the trailing pairs of L and L_n.

Everything runs in float64 with NumPy/SciPy: Householder QR with column
pivoting for the orthonormal bases and LAPACK ``eigh`` for the small
eigenproblem.

Readings where the paper is silent (each is a choice, also listed in the
design notes):

* leading = largest magnitude for the adjacency (Sec. 2 notation), ties broken
  by the larger algebraic value and then by the lower index; for the shifted
  Laplacians leading = largest algebraic value of T (smallest nu of L);
* "orthogonal factor of the QR" of a rank-deficient block is read as a
  rank-revealing QR: columns whose pivoted |R_ii| falls below
  tol * max(1, largest column norm of the block before projection) are dropped;
* the projector (I - Xbar Xbar^T) is applied twice;
* the randomized range finder keeps min(L, numerical rank) singular vectors;
* the Gaussian test matrix Omega is an input;
* Delta of a Laplacian operator is T^(t+1) - pad(T^(t)), including the change
  of the shift alpha on the old block and alpha' on the new block; for the
  normalised Laplacian an isolated node has D^{-1/2}_ii = 0;
* eigenvector signs: the entry of largest magnitude is made positive.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

ADJ, LAP, NLAP = "adj", "lap", "nlap"
G2, G3, RSVD = "g2", "g3", "rsvd"
EXACT, LOWRANK = "exact", "lowrank"

RANK_TOL = 1e-10


class DeltaError(ValueError):
    """A change list that does not follow the transition model of Sec. 2."""


# ------------------------------------------------------------------------------------
# Sec. 2, eq. adj_update: the transition model
# ------------------------------------------------------------------------------------
def adjacency_from_csr(rowptr, col, n=None) -> sp.csr_matrix:
    n = rowptr.shape[0] - 1 if n is None else n
    data = np.ones(col.shape[0], dtype=np.float64)
    return sp.csr_matrix((data, col.astype(np.int64), rowptr.astype(np.int64)), shape=(n, n))


def pad_matrix(M: sp.spmatrix, s: int) -> sp.csr_matrix:
    """The padded matrix: M extended by s identically zero rows and columns (Sec. 2)."""
    n = M.shape[0]
    M = sp.csr_matrix(M)
    return sp.csr_matrix((M.data, M.indices, np.concatenate([M.indptr, np.full(s, M.indptr[-1])])),
                         shape=(n + s, n + s))


def assemble_delta(A: sp.csr_matrix, n_new: int, ei, ej, sign) -> sp.csr_matrix:
    """Delta = [[K, G], [G^T, C]] of eq. adj_update for one step.

    K (old-old) has entries +1 for a new edge and -1 for a removed edge between
    previously existing nodes; G (old-new) and C (new-new) are 0/1.  A change
    list that breaks this definition (insert an existing edge, delete a missing
    one, delete an edge of a new node, self-loop, duplicate, out-of-range id)
    raises DeltaError.
    """
    n = A.shape[0]
    n2 = n + int(n_new)
    ei = np.asarray(ei, dtype=np.int64)
    ej = np.asarray(ej, dtype=np.int64)
    sign = np.asarray(sign, dtype=np.int64)
    if ei.shape != ej.shape or ei.shape != sign.shape:
        raise DeltaError("change arrays differ in length")
    if ei.size:
        if (ei < 0).any() or (ej >= n2).any():
            raise DeltaError("node id out of range")
        if (ei >= ej).any():
            raise DeltaError("each change must have i < j (no self-loops)")
        if not np.isin(sign, [-1, 1]).all():
            raise DeltaError("sign must be +1 or -1")
        key = ei * n2 + ej
        if np.unique(key).size != key.size:
            raise DeltaError("duplicate change")
        old = (ej < n)
        if (sign[~old] < 0).any():
            raise DeltaError("an edge of an appended node can only be inserted")
        present = np.asarray(A[ei[old], ej[old]]).ravel() != 0 if old.any() else np.zeros(0, bool)
        if (present & (sign[old] > 0)).any():
            raise DeltaError("insertion of an existing edge")
        if ((~present) & (sign[old] < 0)).any():
            raise DeltaError("deletion of a missing edge")
    rows = np.concatenate([ei, ej])
    cols = np.concatenate([ej, ei])
    vals = np.concatenate([sign, sign]).astype(np.float64)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n2, n2))


def updated_adjacency(A: sp.csr_matrix, Delta: sp.csr_matrix) -> sp.csr_matrix:
    """A^(t+1) = pad(A^(t)) + Delta (eq. adj_update)."""
    s = Delta.shape[0] - A.shape[0]
    out = (pad_matrix(A, s) + Delta).tocsr()
    out.eliminate_zeros()
    out.sort_indices()
    return out


# ------------------------------------------------------------------------------------
# Sec. 4.2: operators whose leading pairs are tracked
# ------------------------------------------------------------------------------------
def operator_matrix(A: sp.csr_matrix, op: str):
    """The matrix T whose leading eigenpairs are tracked, and its shift.

    adj : T = A (shift 0);
    lap : T = alpha I - L, L = D - A, alpha = 2 d_max  (Sec. 4.2);
    nlap: T_n = 2 I - L_n, L_n = I - D^{-1/2} A D^{-1/2}  (Sec. 4.2), with
          D^{-1/2}_ii = 0 for an isolated node.
    """
    n = A.shape[0]
    if op == ADJ:
        return sp.csr_matrix(A, dtype=np.float64), 0.0
    d = np.asarray(A.sum(axis=1)).ravel()
    if op == LAP:
        alpha = 2.0 * float(d.max()) if n else 0.0
        L = sp.diags(d) - A
        return sp.csr_matrix(alpha * sp.identity(n) - L), alpha
    if op == NLAP:
        s = np.zeros(n)
        nz = d > 0
        s[nz] = 1.0 / np.sqrt(d[nz])
        Ln = sp.identity(n) - sp.diags(s) @ A @ sp.diags(s)
        return sp.csr_matrix(2.0 * sp.identity(n) - Ln), 2.0
    raise ValueError(op)


def operator_delta(A_old, A_new, op):
    """Delta_T = T^(t+1) - pad(T^(t)) (the update of the tracked operator)."""
    T_old, c_old = operator_matrix(A_old, op)
    T_new, c_new = operator_matrix(A_new, op)
    s = A_new.shape[0] - A_old.shape[0]
    DT = (T_new - pad_matrix(T_old, s)).tocsr()
    DT.eliminate_zeros()
    return T_new, DT, c_old, c_new


# ------------------------------------------------------------------------------------
# building blocks
# ------------------------------------------------------------------------------------
def pad_rows(X: np.ndarray, s: int) -> np.ndarray:
    """Xbar = [X; 0_{S x K}] (Alg. 2, padding step)."""
    return np.vstack([X, np.zeros((s, X.shape[1]))])


def project_out(Xbar: np.ndarray, W: np.ndarray, passes: int = 2) -> np.ndarray:
    """(I - Xbar Xbar^T) W, applied ``passes`` times."""
    for _ in range(passes):
        W = W - Xbar @ (Xbar.T @ W)
    return W


def rank_revealing_orth(W: np.ndarray, scale: float, tol: float = RANK_TOL) -> np.ndarray:
    """Orthonormal basis of range(W) from a column-pivoted Householder QR.

    Columns whose |R_ii| <= tol * max(1, scale) are treated as numerically
    dependent and dropped.
    """
    if W.shape[1] == 0:
        return W.copy()
    Q, R, _ = sla.qr(W, mode="economic", pivoting=True)
    diag = np.abs(np.diag(R))
    r = int(np.count_nonzero(diag > tol * max(1.0, scale)))
    return Q[:, :r]


def max_col_norm(W: np.ndarray) -> float:
    return float(np.sqrt((W * W).sum(axis=0)).max()) if W.size else 0.0


def rsvd_basis(Xbar: np.ndarray, D2: sp.csr_matrix, Omega: np.ndarray, L: int,
               tol: float = RANK_TOL) -> np.ndarray:
    """Rank-L randomized basis R of (I - Xbar Xbar^T) Delta_2 (Sec. 3.5, S.1-S.4).

    S.1  Y = (I - Pi) Delta_2 Omega        (Omega: S x (L+P), i.i.d. N(0,1), given)
    S.2  M = orthonormal basis of range(Y); B = M^T (I - Pi) Delta_2 = U S V^T
    S.4  R = M U_L, keeping min(L, numerical rank of B) columns.
    """
    Y = project_out(Xbar, np.asarray(D2 @ Omega))
    M = rank_revealing_orth(Y, max_col_norm(np.asarray(D2 @ Omega)), tol)
    if M.shape[1] == 0:
        return M
    # B = M^T (I - Xbar Xbar^T) Delta_2, evaluated without forming the dense n' x S block
    B = np.asarray((D2.T @ M).T) - (M.T @ Xbar) @ np.asarray((D2.T @ Xbar).T)
    U, sig, _ = np.linalg.svd(B, full_matrices=False)
    keep = int(np.count_nonzero(sig > tol * max(1.0, sig[0] if sig.size else 0.0)))
    return M @ U[:, :min(L, keep)]


def select(theta: np.ndarray, k: int, which: str) -> np.ndarray:
    """Indices of the k leading Ritz values, in output order.

    'LM': largest magnitude first, ties to the larger algebraic value then the
    lower index; 'LA': largest algebraic value first.
    """
    idx = np.arange(theta.size)
    if which == "LM":
        order = np.lexsort((idx, -theta, -np.abs(theta)))
    elif which == "LA":
        order = np.lexsort((idx, -theta))
    else:
        raise ValueError(which)
    return order[:k]


def normalize_signs(X: np.ndarray) -> np.ndarray:
    """Flip each column so that its entry of largest magnitude is positive."""
    if X.size == 0:
        return X
    i = np.argmax(np.abs(X), axis=0)
    s = np.sign(X[i, np.arange(X.shape[1])])
    s[s == 0] = 1.0
    return X * s


def which_for(op: str) -> str:
    return "LM" if op == ADJ else "LA"


# ------------------------------------------------------------------------------------
# Alg. 1 + Alg. 2: one tracking step
# ------------------------------------------------------------------------------------
@dataclasses.dataclass
class StepResult:
    theta: np.ndarray        # K Ritz values of the tracked operator T, leading first
    X: np.ndarray            # n' x K Ritz vectors
    A: sp.csr_matrix         # updated adjacency
    shift: float             # alpha' (lap), 2 (nlap), 0 (adj)
    Z: np.ndarray            # orthonormal projection basis
    H: np.ndarray            # projected matrix
    rank_W: int              # columns kept from the projected augmentation block
    Delta: sp.csr_matrix     # adjacency update
    DeltaT: sp.csr_matrix    # operator update

    op: str = ADJ

    @property
    def nu(self) -> np.ndarray:
        """Eigenvalues of L or L_n (shift - theta); for adj the Ritz values themselves."""
        return self.shift - self.theta if self.op != ADJ else self.theta

    @property
    def nu_rq(self) -> np.ndarray:
        """nu of the Laplacians as the Laplacian quadratic form of the Ritz vectors.

        For a Ritz vector x of T = shift I - L on span(Z), x^T L x = shift - theta
        exactly (Sec. 4.2: nu = alpha - mu); evaluating it as a sum of squared edge
        differences keeps its relative accuracy when nu is small and the shift large."""
        if self.op == ADJ:
            return self.theta
        return laplacian_quadratic_form(self.A, self.X, self.op)


def grest_step(A: sp.csr_matrix, X: np.ndarray, theta_prev: np.ndarray, n_new: int, ei, ej, sign,
               k: int, variant: str = G3, op: str = ADJ, proj: str = EXACT,
               L: Optional[int] = None, Omega: Optional[np.ndarray] = None,
               tol: float = RANK_TOL) -> StepResult:
    """One G-REST update (Alg. 2, one pass of the loop body).

    A          : adjacency at step t (n x n, symmetric, 0/1)
    X, theta_prev : the K tracked pairs of T^(t) (theta in T-space)
    n_new, ei, ej, sign : the update (S appended nodes, changes with i < j)
    variant    : g2 / g3 / rsvd (Table 1 and Sec. 3.5)
    proj       : exact (eq. RR_eigen_graph_upd_main2) or lowrank (eq. ..._main3)
    L, Omega   : RSVD rank and the S x (L+P) Gaussian test matrix
    """
    n = A.shape[0]
    s = int(n_new)
    Delta = assemble_delta(A, s, ei, ej, sign)                       # eq. adj_update
    A_new = updated_adjacency(A, Delta)
    T_new, DT, _, shift = operator_delta(A, A_new, op)
    Xbar = pad_rows(np.asarray(X, dtype=np.float64), s)             # Alg. 2 padding

    V = np.asarray(DT @ Xbar)                                       # Delta Xbar (eq. mat1)
    if variant == G2:
        B2 = np.zeros((n + s, 0))
    elif variant == G3:
        B2 = DT[:, n:].toarray()                                    # Delta_2 (Sec. 3.3)
    elif variant == RSVD:
        if s == 0:
            B2 = np.zeros((n + s, 0))
        else:
            if Omega is None or L is None:
                raise ValueError("rsvd needs L and Omega")
            B2 = rsvd_basis(Xbar, DT[:, n:].tocsr(), np.asarray(Omega, dtype=np.float64), L, tol)
    else:
        raise ValueError(variant)
    W0 = np.hstack([V, B2])
    W = project_out(Xbar, W0)                                        # (I - Pi)[Delta Xbar, B2]
    Q = rank_revealing_orth(W, max_col_norm(W0), tol)
    Z = np.hstack([Xbar, Q])                                        # Alg. 2, basis step

    if proj == EXACT:
        H = Z.T @ np.asarray(T_new @ Z)                              # eq. RR_eigen_graph_upd_main2
    elif proj == LOWRANK:
        C = Z.T @ Xbar
        H = C @ np.diag(np.asarray(theta_prev, dtype=np.float64)) @ C.T + Z.T @ np.asarray(DT @ Z)
    else:
        raise ValueError(proj)
    H = 0.5 * (H + H.T)
    th, F = np.linalg.eigh(H)                                       # Alg. 1, small eigenproblem
    idx = select(th, k, which_for(op))
    Xn = normalize_signs(Z @ F[:, idx])                             # Alg. 2, Ritz vectors
    return StepResult(theta=th[idx].copy(), X=Xn, A=A_new, shift=shift, Z=Z, H=H,
                      rank_W=Q.shape[1], Delta=Delta, DeltaT=DT, op=op)


def laplacian_quadratic_form(A: sp.csr_matrix, X: np.ndarray, op: str) -> np.ndarray:
    """x^T L x = sum over edges (x_i - x_j)^2 (lap), and x^T L_n x = sum over edges
    (x_i/sqrt(d_i) - x_j/sqrt(d_j))^2 + sum over isolated nodes x_i^2 (nlap), per column."""
    C = sp.triu(A, 1).tocoo()
    i, j = C.row, C.col
    X = np.asarray(X, dtype=np.float64)
    if op == LAP:
        D = X[i] - X[j]
        return (D * D).sum(axis=0)
    d = np.asarray(A.sum(axis=1)).ravel()
    s = np.zeros_like(d)
    nz = d > 0
    s[nz] = 1.0 / np.sqrt(d[nz])
    D = X[i] * s[i, None] - X[j] * s[j, None]
    out = (D * D).sum(axis=0)
    iso = ~nz
    if iso.any():
        out = out + (X[iso] ** 2).sum(axis=0)
    return out


# ------------------------------------------------------------------------------------
# drift of tracked pairs (the error proxy behind a restart)
# ------------------------------------------------------------------------------------
def drift_metrics(A: sp.csr_matrix, X: np.ndarray, values: np.ndarray, op: str = ADJ):
    """How far tracked pairs have drifted from eigenpairs of the current graph: the
    measure that decides when to recompute them from scratch, as TIMERS does when its
    accumulated error grows (Sec. 2.2, prior art), with a minimum number of updates
    between recomputations (the setup of Sec. 5).

    orth  = max_ij |(X^T X - I)_ij|
    resid = max_j ||M x_j - values_j x_j||_2 / scale, where M is the matrix whose values
            are reported: A (adj), L (lap), L_n (nlap); scale = max_j |values_j| for the
            adjacency (its norm when the largest-magnitude pair is tracked), and the
            shift of Sec. 4.2 for the Laplacians (2 d_max >= ||L||_2, 2 >= ||L_n||_2).
    """
    X = np.asarray(X, dtype=np.float64)
    values = np.asarray(values, dtype=np.float64)
    k = X.shape[1]
    orth = float(np.abs(X.T @ X - np.eye(k)).max()) if k else 0.0
    T, shift = operator_matrix(A, op)
    if op == ADJ:
        M = T
        scale = float(np.abs(values).max()) if k else 1.0
    else:
        M = shift * sp.identity(A.shape[0]) - T
        scale = shift
    if scale <= 0.0:
        scale = 1.0
    R = M @ X - X * values[None, :]
    resid = float(np.sqrt((R * R).sum(axis=0)).max()) / scale if k else 0.0
    return orth, resid


# ------------------------------------------------------------------------------------
# exact eigenpairs (for method-quality reports and brute-force pins)
# ------------------------------------------------------------------------------------
def leading_eigenpairs(A: sp.csr_matrix, k: int, op: str = ADJ, dense_limit: int = 5000):
    """The exact K leading pairs of T(A): dense eigh for small n, ARPACK otherwise."""
    T, shift = operator_matrix(A, op)
    which = which_for(op)
    n = T.shape[0]
    if n <= dense_limit:
        th, F = np.linalg.eigh(T.toarray())
    else:
        from scipy.sparse.linalg import eigsh
        th, F = eigsh(T, k=min(n - 1, k + 8), which="LM" if which == "LM" else "LA", tol=1e-12)
    idx = select(th, k, which)
    return th[idx].copy(), normalize_signs(F[:, idx]), shift
