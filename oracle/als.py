"""Fast ALS (Appendix C, Algorithm 2) on asymmetric sketches -- test
infrastructure only.

The ALS update of factor A (Appendix C, Eq. (symmetric_als)) is
    A_hat = T_(1) (C kr B) (C^T C o B^T B)^+,
and column r of T_(1) (C kr B) is the contraction T(I, b_r, c_r) (the
Khatri-Rao identity quoted there).  Each such contraction is estimated per
sketch by Proposition 1 with the two count sketches taken of two different
vectors, and the estimate is the median over the B sketches.  B and C follow
with the roles of the modes rotated.  After every update lambda_r is the
column norm and the column is normalised.

Readings (the paper is silent or at odds with itself):
  * Algorithm 2 as printed sets A_hat to the median estimates alone; the
    appendix's update equation multiplies them by the k x k pseudo-inverse of
    (C^T C o B^T B).  Both are the same when the other factors have orthonormal
    columns; we follow the equation (the textbook ALS update);
  * the pseudo-inverse drops eigenvalues below 1e-12 times the largest;
  * the factors are held as rows: A[r] is column r of the paper's A;
  * lambda after a sweep is the norm from the last (C) update.
Parity pinned by: the injective-hash special case (each estimate is then the
exact contraction, and sketched ALS is exact ALS); unbiasedness of the
two-vector estimate by full enumeration of hash and sign draws; exact ALS
recovering an exactly low-rank tensor.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .sketch import count_sketch
from .contract import median


def contract_two(sT: np.ndarray, h, xi, X: np.ndarray, Y: np.ndarray, rd: int) -> np.ndarray:
    """One sketch's estimate of the contraction of T with X in mode (rd+1)%3
    and Y in mode (rd+2)%3, read off in mode rd (Proposition 1 with the two
    count sketches of different vectors):
        sbar = F^{-1}( F(s_T) o conj F(s_a X) o conj F(s_b Y) ),
        v_i  = xi_rd(i) sbar[h_rd(i)].
    X, Y: [..., n]; returns [..., n]."""
    b = sT.shape[-1]
    a, c = (rd + 1) % 3, (rd + 2) % 3
    S = np.fft.rfft(sT)
    SX = np.fft.rfft(count_sketch(X, h[a], xi[a], b), axis=-1)
    SY = np.fft.rfft(count_sketch(Y, h[c], xi[c], b), axis=-1)
    sbar = np.fft.irfft(S * np.conj(SX) * np.conj(SY), n=b, axis=-1)
    return np.asarray(xi[rd], dtype=np.float64) * sbar[..., np.asarray(h[rd], dtype=np.int64)]


def contract_two_dense(T: np.ndarray, X: np.ndarray, Y: np.ndarray, rd: int) -> np.ndarray:
    """The exact contraction the estimate targets: T(I, x, y), T(y, I, x) or
    T(x, y, I) for rd = 0, 1, 2 (x in mode rd+1, y in mode rd+2, cyclically).
    X, Y: [k][n]; returns [k][n]."""
    if rd == 0:
        return np.einsum("ijk,rj,rk->ri", T, X, Y)
    if rd == 1:
        return np.einsum("ijk,rk,ri->rj", T, X, Y)
    return np.einsum("ijk,ri,rj->rk", T, X, Y)


def pinv_sym(G: np.ndarray, rcond: float = 1e-12) -> np.ndarray:
    """Pseudo-inverse of a symmetric matrix (numpy's SVD-based routine)."""
    return np.linalg.pinv(G, rcond=rcond, hermitian=True)


def als_update(V: np.ndarray, X: np.ndarray, Y: np.ndarray):
    """One factor update from the contraction estimates V [k][n] (rows
    T(I, x_r, y_r)) and the other two factors X, Y [k][n]:
    A_hat = G^+ V with G = (X X^T) o (Y Y^T); returns (lambda, unit rows)."""
    G = (X @ X.T) * (Y @ Y.T)
    A = pinv_sym(G) @ V
    lam = np.linalg.norm(A, axis=1)
    return lam, A / np.where(lam > 0, lam, 1.0)[:, None]


@dataclasses.dataclass
class AlsResult:
    lam: np.ndarray        # [k]
    F: np.ndarray          # [3][k][n] unit rows of A, B, C


def als_sketched(S: np.ndarray, h, xi, k: int, T: int, F0: np.ndarray) -> AlsResult:
    """Algorithm 2 (with the update equation's pseudo-inverse).  S: [B][b]
    time-domain sketches, h/xi: [B][3][n], F0: [3][k][n] initial rows."""
    F = np.array(F0, dtype=np.float64, copy=True)
    B = S.shape[0]
    lam = np.zeros(k)
    for _ in range(T):
        for rd in range(3):
            X, Y = F[(rd + 1) % 3], F[(rd + 2) % 3]
            V = np.stack([contract_two(S[m], h[m], xi[m], X, Y, rd) for m in range(B)], axis=1)
            lam, F[rd] = als_update(median(V, axis=1), X, Y)
    return AlsResult(lam=lam, F=F)


def als_dense(Tt: np.ndarray, k: int, T: int, F0: np.ndarray) -> AlsResult:
    """The same iteration with exact contractions (plain ALS)."""
    F = np.array(F0, dtype=np.float64, copy=True)
    lam = np.zeros(k)
    for _ in range(T):
        for rd in range(3):
            X, Y = F[(rd + 1) % 3], F[(rd + 2) % 3]
            lam, F[rd] = als_update(contract_two_dense(Tt, X, Y, rd), X, Y)
    return AlsResult(lam=lam, F=F)
