"""Dense brute-force forms of the paper's equations, for tiny tensors.

Used only to pin the oracle.  Everything here is written from the matrix
formulas of Section II (unfolding, Khatri-Rao, eq. gradient_F, eq.
hessian_F) with dense masks, not from the oracle's row-wise loops.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np


def khatri_rao(mats: Sequence[np.ndarray]) -> np.ndarray:
    """Column-wise Kronecker product A_1 (.) A_2 (.) ... (first factor slowest)."""
    out = mats[0]
    for M in mats[1:]:
        R = out.shape[1]
        out = (out[:, None, :] * M[None, :, :]).reshape(-1, R)
    return out


def unfold(T: np.ndarray, mode: int) -> np.ndarray:
    """Mode-i unfolding whose column index runs over the remaining modes with
    the lowest-numbered one fastest, matching
    Y_(i) = U^(i) (U^(N) (.) ... (.) U^(i+1) (.) U^(i-1) (.) ... (.) U^(1))^T."""
    N = T.ndim
    rest = [m for m in range(N) if m != mode]
    # Fortran order over `rest` = first remaining mode varies fastest
    return np.transpose(T, [mode] + rest).reshape(T.shape[mode], -1, order="F")


def kr_for_mode(U: Sequence[np.ndarray], mode: int) -> np.ndarray:
    """K^(i) = U^(N) (.) ... (.) U^(i+1) (.) U^(i-1) (.) ... (.) U^(1)."""
    rest = [m for m in range(len(U)) if m != mode]
    return khatri_rao([U[m] for m in reversed(rest)])


def cpd_full(U: Sequence[np.ndarray]) -> np.ndarray:
    """[[U^(1), ..., U^(N)]] as a dense array (eq. Xo_densef)."""
    R = U[0].shape[1]
    T = np.zeros(tuple(u.shape[0] for u in U))
    for r in range(R):
        t = U[0][:, r]
        for u in U[1:]:
            t = np.multiply.outer(t, u[:, r])
        T += t
    return T


def dense_data(dims, coords: np.ndarray, values: np.ndarray):
    """Dense X and mask M from COO."""
    X = np.zeros(dims)
    M = np.zeros(dims)
    idx = tuple(coords[:, m] for m in range(coords.shape[1]))
    X[idx] = values.astype(np.float64)
    M[idx] = 1.0
    return X, M


def nmc_gradient(X: np.ndarray, M: np.ndarray, A: np.ndarray, B: np.ndarray, lam: float) -> np.ndarray:
    """eq. gradient_F: -(M*X - M*(A B^T)) B + lam A."""
    return -(M * X - M * (A @ B.T)) @ B + lam * A


def nmc_hessian(M: np.ndarray, B: np.ndarray, lam: float) -> np.ndarray:
    """eq. hessian_F: (B^T kron I_P) diag(vec M) (B kron I_P) + lam I_{PR}, in
    the column-major vec(A) ordering (index r*P + p)."""
    P = M.shape[0]
    R = B.shape[1]
    BI = np.kron(B, np.eye(P))                      # (Q P) x (R P)
    vecM = M.reshape(-1, order="F")                 # column-major vec
    return BI.T @ (vecM[:, None] * BI) + lam * np.eye(P * R)


def nmc_objective(X, M, A, B, lam):
    """eq. matrix_NMC."""
    return 0.5 * np.sum((M * (X - A @ B.T)) ** 2) + 0.5 * lam * np.sum(A ** 2)


def ntc_objective(dims, coords, values, U, lam):
    """eq. Problem_TC on the observed set."""
    X, M = dense_data(dims, coords, values)
    return 0.5 * np.sum((M * (X - cpd_full(U))) ** 2) + 0.5 * lam * sum(np.sum(u ** 2) for u in U)


def row_lmax(Hrow: np.ndarray) -> float:
    return float(np.linalg.eigvalsh(Hrow).max())


def full_batch_mode_update(X, M, U: List[np.ndarray], mode: int, lam: float, max_inner: int) -> np.ndarray:
    """Alg. 1 with the whole observed set as the minibatch (c = 1), dense:
    every row p uses its own L_p = max eig of its Hessian block, which for the
    row-major layout is B^T diag(M(p,:)) B + lam I."""
    Xi = unfold(X, mode)
    Mi = unfold(M, mode)
    B = kr_for_mode(U, mode)
    A = U[mode].copy()
    Y = A.copy()
    P, R = A.shape
    Ls = np.array([row_lmax(B.T @ (Mi[p][:, None] * B) + lam * np.eye(R)) for p in range(P)])
    active = Mi.sum(axis=1) > 0
    for _ in range(max_inner):
        G = nmc_gradient(Xi, Mi, Y, B, lam)
        An = np.maximum(0.0, Y - G / Ls[:, None])
        beta = (np.sqrt(Ls) - np.sqrt(lam)) / (np.sqrt(Ls) + np.sqrt(lam))
        Yn = An + beta[:, None] * (An - A)
        An[~active] = A[~active]
        Yn[~active] = Y[~active]
        A, Y = An, Yn
    return A
