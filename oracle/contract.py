"""Sketched tensor contractions (oracle side) -- test infrastructure only.

T(I,u,u) is read off the FFT output by Proposition 1; T(u,u,u) is the sketch
inner product of Eq. (3) with X = u (x) u (x) u.  The DFT convention is the
unnormalised forward transform F(x)_k = sum_t x_t e^{-2 pi i k t / b} and the
inverse carries the 1/b, under which Proposition 1 holds exactly as printed.
"""
from __future__ import annotations

import numpy as np

from .sketch import count_sketch, circular_convolution, circular_convolution_fft


def median(x: np.ndarray, axis: int) -> np.ndarray:
    """Median over the B sketches (Algorithm 1).  For even B it is the mean of
    the two middle order statistics (the paper does not fix this case)."""
    return np.median(x, axis=axis)


def power_update_sketch(sT: np.ndarray, h, xi, U: np.ndarray) -> np.ndarray:
    """One sketch's estimate of T(I,u,u) by Proposition 1:
        sbar = F^{-1}( F(s_T) o conj F(s_{2,u}) o conj F(s_{3,u}) )
        v_i  = xi_1(i) * sbar[h_1(i)]
    ``U`` is [..., n]; returns [..., n]."""
    b = sT.shape[-1]
    S = np.fft.rfft(sT)
    S2 = np.fft.rfft(count_sketch(U, h[1], xi[1], b), axis=-1)
    S3 = np.fft.rfft(count_sketch(U, h[2], xi[2], b), axis=-1)
    sbar = np.fft.irfft(S * np.conj(S2) * np.conj(S3), n=b, axis=-1)
    return np.asarray(xi[0], dtype=np.float64) * sbar[..., np.asarray(h[0], dtype=np.int64)]


def power_update_direct(sT: np.ndarray, h, xi, u: np.ndarray) -> np.ndarray:
    """The quantity Proposition 1 computes, from its left-hand side:
        v_i = < s_T , s_{1,e_i} * s_{2,u} * s_{3,u} >
    with the convolutions done directly (O(b^2)); small b only."""
    b = sT.shape[-1]
    n = u.shape[-1]
    s2 = count_sketch(u, h[1], xi[1], b)
    s3 = count_sketch(u, h[2], xi[2], b)
    c23 = circular_convolution(s2, s3)
    v = np.zeros(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        s1 = count_sketch(e, h[0], xi[0], b)
        v[i] = float(np.dot(sT, circular_convolution(s1, c23)))
    return v


def tuuu_sketch(sT: np.ndarray, h, xi, U: np.ndarray) -> np.ndarray:
    """One sketch's estimate of T(u,u,u) = <T, u(x)u(x)u> by Eq. (3): the
    sketch inner product <s_T, s_{1,u} * s_{2,u} * s_{3,u}>, with the rank-1
    sketch formed by Eq. (2) through FFTs.  ``U`` is [..., n]."""
    b = sT.shape[-1]
    s1 = count_sketch(U, h[0], xi[0], b)
    s2 = count_sketch(U, h[1], xi[1], b)
    s3 = count_sketch(U, h[2], xi[2], b)
    sX = circular_convolution_fft(circular_convolution_fft(s1, s2), s3)
    return np.sum(sX * sT, axis=-1)


def tuuu_direct(sT: np.ndarray, h, xi, u: np.ndarray) -> float:
    """Eq. (3) with the rank-1 sketch by direct convolution; small b only."""
    b = sT.shape[-1]
    s1 = count_sketch(u, h[0], xi[0], b)
    s2 = count_sketch(u, h[1], xi[1], b)
    s3 = count_sketch(u, h[2], xi[2], b)
    return float(np.dot(sT, circular_convolution(circular_convolution(s1, s2), s3)))


def power_update(S: np.ndarray, h, xi, U: np.ndarray):
    """One power step of Algorithm 1 for all restarts at once.

    S: [B][b] sketches; h, xi: [B][3][n]; U: [L][n] current vectors.
    Returns (V [L][B][n] per-sketch estimates, Unew [L][n], flags [L]).
    vbar_i = med_m Re v_i^(m); u <- vbar / ||vbar||.  When ||vbar|| is zero or
    not finite the vector is kept and the restart's flag is set (the paper is
    silent on this case)."""
    B = S.shape[0]
    L = U.shape[0]
    V = np.stack([power_update_sketch(S[m], h[m], xi[m], U) for m in range(B)], axis=1)
    vbar = median(V, axis=1)
    Unew = U.copy()
    flags = np.zeros(L, dtype=np.int32)
    for tau in range(L):
        nrm = float(np.linalg.norm(vbar[tau]))
        if nrm > 0.0 and np.isfinite(nrm):
            Unew[tau] = vbar[tau] / nrm
        else:
            flags[tau] = 1
    return V, Unew, flags


def contract_uuu(S: np.ndarray, h, xi, U: np.ndarray):
    """Selection estimates of Algorithm 1: lambda_tau^(m) ~ T(u_tau,u_tau,u_tau)
    from sketch m, and lambda_tau = med_m lambda_tau^(m).
    Returns (lam_per [L][B], lam_med [L])."""
    B = S.shape[0]
    lam_per = np.stack([tuuu_sketch(S[m], h[m], xi[m], U) for m in range(B)], axis=1)
    return lam_per, median(lam_per, axis=1)
