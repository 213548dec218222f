"""Gradients of sketched objectives (oracle side) -- test infrastructure only.

Two differentiable objectives are built from the sketch inner product of
Eq. (3) and the linearity of the sketch (Section 3.1):

  f^(m)(u)    = < s^(m)(T), s_1^(m)(u) * s_2^(m)(u) * s_3^(m)(u) >   (T(u,u,u) from sketch m)
  f(u)        = med_m f^(m)(u)
  loss(lam,U) = (1/B) sum_m || s^(m)(T) - sum_i lam_i s^(m)(u_i (x) u_i (x) u_i) ||^2

Each count sketch s_j(u) is linear in u with d s_j(u)[t] / d u_i =
xi_j(i) [h_j(i) == t], so the derivative of the triple product through mode j
is a circular correlation of the other sketch with the convolution of the
remaining two count sketches, read at h_j(i) -- the read-off of
Proposition 1 with mode j in the place of mode 1.  The median's derivative is
that of the sketch it selects (for even B the mean of the two middle ones,
ranks breaking ties by sketch index).

Parity unpinned beyond the pins in tests/test_oracle_grad_pins.py (central
finite differences and the injective-hash reduction to the dense gradient).
"""
from __future__ import annotations

import numpy as np

from .sketch import count_sketch, circular_convolution, circular_convolution_fft

_OTHER = {0: (1, 2), 1: (0, 2), 2: (0, 1)}


def read_off_mode(s: np.ndarray, h, xi, U: np.ndarray, j: int) -> np.ndarray:
    """g_i = xi_j(i) * corr(s, s_a(u) * s_b(u))[h_j(i)] for the two modes a, b
    other than j, through FFTs (Proposition 1 with the modes permuted).
    ``s`` is one time-domain sketch [b]; ``U`` is [..., n]."""
    a, c = _OTHER[j]
    b = s.shape[-1]
    S = np.fft.rfft(s)
    Sa = np.fft.rfft(count_sketch(U, h[a], xi[a], b), axis=-1)
    Sb = np.fft.rfft(count_sketch(U, h[c], xi[c], b), axis=-1)
    corr = np.fft.irfft(S * np.conj(Sa) * np.conj(Sb), n=b, axis=-1)
    return np.asarray(xi[j], dtype=np.float64) * corr[..., np.asarray(h[j], dtype=np.int64)]


def read_off_mode_direct(s: np.ndarray, h, xi, u: np.ndarray, j: int) -> np.ndarray:
    """The same quantity from its definition, the derivative of the triple
    product along mode j: g_i = < s, s_j(e_i) * s_a(u) * s_b(u) >, with the
    convolutions done directly (small b only)."""
    a, c = _OTHER[j]
    b = s.shape[-1]
    n = u.shape[-1]
    cab = circular_convolution(count_sketch(u, h[a], xi[a], b), count_sketch(u, h[c], xi[c], b))
    g = np.zeros(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        g[i] = float(np.dot(s, circular_convolution(count_sketch(e, h[j], xi[j], b), cab)))
    return g


def triple_product(s: np.ndarray, h, xi, U: np.ndarray) -> np.ndarray:
    """f(u) = < s, s_1(u) * s_2(u) * s_3(u) > for every row of U."""
    b = s.shape[-1]
    s1 = count_sketch(U, h[0], xi[0], b)
    s2 = count_sketch(U, h[1], xi[1], b)
    s3 = count_sketch(U, h[2], xi[2], b)
    return np.sum(s * circular_convolution_fft(circular_convolution_fft(s1, s2), s3), axis=-1)


def triple_product_grad(s: np.ndarray, h, xi, U: np.ndarray) -> np.ndarray:
    """d f / d u = sum over the three modes of read_off_mode."""
    return sum(read_off_mode(s, h, xi, U, j) for j in range(3))


def median_members(values: np.ndarray):
    """Indices whose mean is the median of ``values`` (1-D): the element of
    rank (B-1)/2 for odd B, the two middle ranks for even B; ranks break ties
    by index (a stable sort)."""
    order = np.argsort(values, kind="stable")
    B = len(values)
    if B % 2:
        return [int(order[(B - 1) // 2])]
    return [int(order[B // 2 - 1]), int(order[B // 2])]


def tuuu_with_grad(S: np.ndarray, h, xi, U: np.ndarray):
    """f(u) = med_m f^(m)(u) and its gradient for every row of U.

    S: [B][b] time-domain sketches; h, xi: [B][3][n]; U: [L][n].
    Returns (f_med [L], f_per [L][B], grad [L][n])."""
    B = S.shape[0]
    f_per = np.stack([triple_product(S[m], h[m], xi[m], U) for m in range(B)], axis=1)
    g_per = np.stack([triple_product_grad(S[m], h[m], xi[m], U) for m in range(B)], axis=1)
    L = U.shape[0]
    f_med = np.median(f_per, axis=1)
    grad = np.zeros_like(U, dtype=np.float64)
    for tau in range(L):
        sel = median_members(f_per[tau])
        grad[tau] = np.mean([g_per[tau, m] for m in sel], axis=0)
    return f_med, f_per, grad


def cp_residual(S: np.ndarray, h, xi, lam: np.ndarray, U: np.ndarray) -> np.ndarray:
    """r^(m) = s^(m)(T) - sum_i lam_i s^(m)(u_i^{(x)3}), each rank-1 sketch by
    Eq. (2) (convolution of the three count sketches)."""
    B, b = S.shape
    R = S.astype(np.float64).copy()
    for m in range(B):
        s1 = count_sketch(U, h[m][0], xi[m][0], b)
        s2 = count_sketch(U, h[m][1], xi[m][1], b)
        s3 = count_sketch(U, h[m][2], xi[m][2], b)
        R[m] -= np.asarray(lam, dtype=np.float64) @ circular_convolution_fft(
            circular_convolution_fft(s1, s2), s3)
    return R


def cp_loss(S: np.ndarray, h, xi, lam: np.ndarray, U: np.ndarray) -> float:
    """loss = (1/B) sum_m ||r^(m)||^2."""
    R = cp_residual(S, h, xi, lam, U)
    return float(np.sum(R * R) / S.shape[0])


def cp_loss_grad(S: np.ndarray, h, xi, lam: np.ndarray, U: np.ndarray):
    """Gradient of cp_loss:
        d loss / d lam_i = -(2/B) sum_m < r^(m), s^(m)(u_i^{(x)3}) >
        d loss / d u_i   = -(2/B) lam_i sum_m sum_j read_off_mode(r^(m), u_i, j).
    Returns (loss, grad_lam [k], grad_U [k][n])."""
    B = S.shape[0]
    R = cp_residual(S, h, xi, lam, U)
    loss = float(np.sum(R * R) / B)
    g_lam = np.zeros(len(lam))
    g_U = np.zeros(U.shape)
    for m in range(B):
        g_lam += triple_product(R[m], h[m], xi[m], U)
        g_U += triple_product_grad(R[m], h[m], xi[m], U)
    g_lam *= -2.0 / B
    g_U *= (-2.0 / B) * np.asarray(lam, dtype=np.float64)[:, None]
    return loss, g_lam, g_U
