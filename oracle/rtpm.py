"""Robust tensor power method, sketched (Algorithm 1) and plain -- test
infrastructure only.

Readings taken where the paper is silent:
  * lambda_hat is evaluated at u_hat = u_T^(tau*) / ||u_T^(tau*)|| (a no-op up
    to rounding when u_T is already unit length), as the median over sketches
    of <s^(m), s^(m)(u_hat^{(x)3})>;
  * argmax ties go to the lowest restart index; a non-finite lambda_tau never
    wins;
  * a restart whose median vector is zero or not finite keeps its vector and is
    flagged.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .contract import median, power_update, contract_uuu, tuuu_sketch
from .sketch import sketch_rank1_fft
from .dense import dense_TIuu


@dataclasses.dataclass
class RtpmResult:
    lam: np.ndarray        # [k] recovered eigenvalues
    U: np.ndarray          # [k][n] recovered unit vectors
    tau: np.ndarray        # [k] selected restart
    flags: np.ndarray      # [k][L] restarts that hit a zero/non-finite update
    lam_tau: np.ndarray    # [k][L] selection values lambda_tau
    S: np.ndarray | None   # deflated sketches [B][b] (sketched method only)


def _select(lam_tau: np.ndarray) -> int:
    key = np.where(np.isfinite(lam_tau), lam_tau, -np.inf)
    return int(np.argmax(key))          # first maximum = lowest tau


def rtpm_sketched(S: np.ndarray, h, xi, k: int, L: int, T: int,
                  u0: np.ndarray) -> RtpmResult:
    """Algorithm 1 on precomputed sketches S [B][b] with tables h, xi [B][3][n]
    and start vectors u0 [k][L][n].  Sketches are reused across all
    contractions (built once, as in the algorithm's initialisation)."""
    S = np.array(S, dtype=np.float64, copy=True)
    B, b = S.shape
    n = u0.shape[-1]
    lam_out = np.zeros(k)
    U_out = np.zeros((k, n))
    tau_out = np.zeros(k, dtype=np.int64)
    flag_out = np.zeros((k, L), dtype=np.int32)
    lam_tau_out = np.zeros((k, L))
    for c in range(k):
        U = np.array(u0[c], dtype=np.float64, copy=True)
        for _ in range(T):
            _, U, f = power_update(S, h, xi, U)
            flag_out[c] |= f
        _, lam_tau = contract_uuu(S, h, xi, U)
        tau = _select(lam_tau)
        u_hat = U[tau] / np.linalg.norm(U[tau])
        lam_hat = float(median(np.array([tuuu_sketch(S[m], h[m], xi[m], u_hat)
                                         for m in range(B)]), axis=0))
        # Deflation: subtract the sketch of lam_hat * u_hat^{(x)3}, same tables.
        for m in range(B):
            S[m] -= lam_hat * sketch_rank1_fft(u_hat, u_hat, u_hat, h[m], xi[m], b)
        lam_out[c], U_out[c], tau_out[c] = lam_hat, u_hat, tau
        lam_tau_out[c] = lam_tau
    return RtpmResult(lam=lam_out, U=U_out, tau=tau_out, flags=flag_out,
                      lam_tau=lam_tau_out, S=S)


def rtpm_dense(T: np.ndarray, k: int, L: int, Titer: int, u0: np.ndarray) -> RtpmResult:
    """The plain robust tensor power method on the dense tensor (Section 2):
    same start vectors, selection and deflation, exact contractions."""
    T = np.array(T, dtype=np.float64, copy=True)
    n = T.shape[0]
    lam_out = np.zeros(k)
    U_out = np.zeros((k, n))
    tau_out = np.zeros(k, dtype=np.int64)
    flag_out = np.zeros((k, L), dtype=np.int32)
    lam_tau_out = np.zeros((k, L))
    for c in range(k):
        U = np.array(u0[c], dtype=np.float64, copy=True)
        for tau in range(L):
            for _ in range(Titer):
                v = dense_TIuu(T, U[tau])
                nrm = float(np.linalg.norm(v))
                if nrm > 0.0 and np.isfinite(nrm):
                    U[tau] = v / nrm
                else:
                    flag_out[c, tau] = 1
        lam_tau = np.array([float(U[t] @ dense_TIuu(T, U[t])) for t in range(L)])
        tau = _select(lam_tau)
        u_hat = U[tau] / np.linalg.norm(U[tau])
        lam_hat = float(u_hat @ dense_TIuu(T, u_hat))
        T -= lam_hat * np.einsum("i,j,k->ijk", u_hat, u_hat, u_hat)
        lam_out[c], U_out[c], tau_out[c] = lam_hat, u_hat, tau
        lam_tau_out[c] = lam_tau
    return RtpmResult(lam=lam_out, U=U_out, tau=tau_out, flags=flag_out,
                      lam_tau=lam_tau_out, S=None)
