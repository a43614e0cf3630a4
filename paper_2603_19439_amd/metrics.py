"""Accuracy measures for comparing two sets of tracked eigenpairs.

All functions take plain NumPy arrays and compute in float64.  They compare any
two results (GPU vs oracle, or either vs exact eigenpairs); none of them is part
of the update itself.
"""
from __future__ import annotations

import numpy as np


def eig_rel_error(theta: np.ndarray, ref: np.ndarray) -> float:
    """max_j |theta_j - ref_j| / max(|ref_j|, 1e-8 * max_i |ref_i|)."""
    theta = np.asarray(theta, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.size == 0:
        return 0.0
    floor = 1e-8 * np.abs(ref).max()
    den = np.maximum(np.abs(ref), max(floor, np.finfo(float).tiny))
    return float(np.max(np.abs(theta - ref) / den))


def gap_prefix(ref_all: np.ndarray, k: int, rel_gap: float = 1e-3, scale: float = None) -> int:
    """Largest k* <= k whose cut is separated: |ref_{k*} - ref_{k*+1}| >= rel_gap * scale,
    with scale = |ref_1| unless given.

    ``ref_all`` lists the reference values in output order (at least k+1 of them if a
    (k+1)-th value is known)."""
    ref_all = np.asarray(ref_all, dtype=np.float64)
    if scale is None:
        scale = max(abs(ref_all[0]), 1e-300) if ref_all.size else 1.0
    for kk in range(min(k, ref_all.size - 1), 0, -1):
        if abs(ref_all[kk - 1] - ref_all[kk]) >= rel_gap * scale:
            return kk
    return k if ref_all.size <= k else 0


def subspace_sine(U: np.ndarray, V: np.ndarray) -> float:
    """||(I - V V^T) U||_2 for orthonormal U, V (sine of the largest principal angle).

    Computed from the residual itself, not from 1 - cos^2, so that angles near
    machine precision are resolved."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    if U.shape[1] == 0:
        return 0.0
    R = U - V @ (V.T @ U)
    return float(np.linalg.norm(R, 2))


def orthonormality(U: np.ndarray) -> float:
    U = np.asarray(U, dtype=np.float64)
    return float(np.abs(U.T @ U - np.eye(U.shape[1])).max())


def residual(T, U: np.ndarray, theta: np.ndarray, norm_T: float) -> float:
    """max_j ||T u_j - theta_j u_j||_2 / ||T||_2 (T any matrix-like with @)."""
    U = np.asarray(U, dtype=np.float64)
    R = np.asarray(T @ U) - U * np.asarray(theta, dtype=np.float64)[None, :]
    return float(np.sqrt((R * R).sum(axis=0)).max() / max(norm_T, 1e-300))


def psi_angles(X_ref: np.ndarray, X_est: np.ndarray) -> np.ndarray:
    """Per-vector angles arccos(|x_ref^T x_est|) between unit vectors."""
    a = np.abs(np.einsum("ij,ij->j", X_ref / np.linalg.norm(X_ref, axis=0),
                         X_est / np.linalg.norm(X_est, axis=0)))
    return np.arccos(np.clip(a, 0.0, 1.0))
