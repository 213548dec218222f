"""Dense (exact) contractions and recovery metrics -- test infrastructure only.

T(u,u,u) = sum_ijk T_ijk u_i u_j u_k and T(I,u,u)_i = sum_jk T_ijk u_j u_k
(Section 2).  Residual is the rank-k CP objective ||T - sum_i lam_i v_i^{(x)3}||_F^2
(Section 2); a recovered vector counts as wrong when no planted vector is
within squared distance 0.1 of it (Section 5.1, Table 3 caption).
"""
from __future__ import annotations

import numpy as np


def dense_TIuu(T: np.ndarray, u: np.ndarray) -> np.ndarray:
    return np.einsum("ijk,j,k->i", np.asarray(T, dtype=np.float64), u, u)


def dense_Tuuu(T: np.ndarray, u: np.ndarray) -> float:
    return float(np.einsum("ijk,i,j,k->", np.asarray(T, dtype=np.float64), u, u, u))


def residual_dense(T: np.ndarray, lam: np.ndarray, V: np.ndarray) -> float:
    """||T - sum_i lam_i v_i^{(x)3}||_F^2 with the tensor formed explicitly."""
    R = np.asarray(T, dtype=np.float64).copy()
    for i in range(len(lam)):
        R -= lam[i] * np.einsum("i,j,k->ijk", V[i], V[i], V[i])
    return float(np.sum(R * R))


def residual_factored(lam_true, A_true, lam_hat, V_hat) -> float:
    """The same squared residual for a tensor given by factors, expanded with
    <a(x)a(x)a, c(x)c(x)c> = (a.c)^3 so the tensor is never formed."""
    G11 = (A_true @ A_true.T) ** 3
    G12 = (A_true @ V_hat.T) ** 3
    G22 = (V_hat @ V_hat.T) ** 3
    return float(lam_true @ G11 @ lam_true - 2.0 * lam_true @ G12 @ lam_hat
                 + lam_hat @ G22 @ lam_hat)


def wrong_vectors(V_true: np.ndarray, V_hat: np.ndarray, thresh: float = 0.1) -> int:
    """Number of planted vectors with no recovered vector within ||v - v_hat||^2 <= thresh."""
    d2 = ((V_true[:, None, :] - V_hat[None, :, :]) ** 2).sum(-1)
    return int(np.sum(d2.min(axis=1) > thresh))
