"""Loss-of-orthogonality and Arnoldi-relation measures, in NumPy FP64.

TEST INFRASTRUCTURE ONLY (part of the oracle package). These read a basis V and
a Hessenberg matrix H, wherever they came from, and compute the quantities the
paper uses to judge a Gram-Schmidt scheme.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def strict_lower_gram(V: np.ndarray) -> np.ndarray:
    """L with V^T V = I + L + L^T, L strictly lower triangular (Section II)."""
    G = V.T @ V
    return np.tril(G, -1)


def t_from_basis(V: np.ndarray) -> np.ndarray:
    """T = (I + L^T)^{-1} formed from an explicit Gram matrix (Malard-Paige form, Section II)."""
    k = V.shape[1]
    L = strict_lower_gram(V)
    return np.linalg.solve(np.eye(k) + L.T, np.eye(k))


def paige_s_norm(T: np.ndarray) -> float:
    """Paige's ||S||_2 with S = (I + L^T)^{-1} L^T = I - T (Section II)."""
    k = T.shape[0]
    if k == 0:
        return 0.0
    return float(np.linalg.norm(np.eye(k) - T, 2))


def s_norm_history(T: np.ndarray, j: int) -> np.ndarray:
    """||S_k||_2 for the leading k x k blocks, k = 1..j+1 (T is built one column per step)."""
    return np.array([paige_s_norm(T[:k, :k]) for k in range(1, j + 2)])


def orth_loss(V: np.ndarray) -> float:
    """||I - V^T V||_2."""
    k = V.shape[1]
    return float(np.linalg.norm(np.eye(k) - V.T @ V, 2))


def orth_loss_history(V: np.ndarray, j: int) -> np.ndarray:
    """||I - V_k^T V_k||_2 for k = 1..j."""
    G = V[:, :j].T @ V[:, :j]
    return np.array([float(np.linalg.norm(np.eye(k) - G[:k, :k], 2)) for k in range(1, j + 1)])


def arnoldi_residual(A, V: np.ndarray, H: np.ndarray, j: int) -> float:
    """||A V_j - V_{j+1} H_j||_F / (||A||_F (j+1)) (Section III, Arnoldi relation)."""
    A = sp.csr_matrix(A)
    AV = A @ V[:, :j]
    E = AV - V[:, : j + 1] @ H[: j + 1, :j]
    return float(np.linalg.norm(E) / (spla.norm(A) * (j + 1)))
