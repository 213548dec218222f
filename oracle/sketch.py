"""Count sketch and tensor sketch (oracle side) -- test infrastructure only.

Indices are 0-based as in the paper's notation appendix: a length-b sketch is
(s_0, ..., s_{b-1}) and circular convolution is
    (a * c)_t = sum over (i + j) mod b == t of a_i c_j.
"""
from __future__ import annotations

import numpy as np


def count_sketch(u: np.ndarray, h: np.ndarray, xi: np.ndarray, b: int) -> np.ndarray:
    """Count sketch s_u(t) = sum_{h(i)=t} xi(i) u_i (Section 3.1).

    ``u`` may carry leading batch axes; the sketch is taken over the last."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros(u.shape[:-1] + (b,), dtype=np.float64)
    for i in range(u.shape[-1]):
        out[..., int(h[i])] += float(xi[i]) * u[..., i]
    return out


def sketch_dense(T: np.ndarray, h: np.ndarray, xi: np.ndarray, b: int) -> np.ndarray:
    """Tensor sketch of a dense n x n x n tensor by Eq. (1):
        s_T(t) = sum over H(i,j,k) == t of xi_1(i) xi_2(j) xi_3(k) T_ijk,
        H(i,j,k) = (h_1(i) + h_2(j) + h_3(k)) mod b.
    ``h``/``xi`` are [3][n] (one sketch).  Every entry is scattered once."""
    T = np.asarray(T, dtype=np.float64)
    n = T.shape[0]
    h1, h2, h3 = (np.asarray(h[j], dtype=np.int64) for j in range(3))
    x1, x2, x3 = (np.asarray(xi[j], dtype=np.float64) for j in range(3))
    s = np.zeros(b, dtype=np.float64)
    for i in range(n):
        H = (h1[i] + h2[:, None] + h3[None, :]) % b
        W = x1[i] * x2[:, None] * x3[None, :] * T[i]
        np.add.at(s, H.ravel(), W.ravel())
    return s


def circular_convolution(a: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Direct O(b^2) circular convolution (notation appendix)."""
    b = a.shape[-1]
    out = np.zeros(np.broadcast_shapes(a.shape, c.shape), dtype=np.float64)
    for i in range(b):
        # a_i contributes a_i * c_j to index (i + j) mod b, i.e. c rolled by i.
        out += a[..., i:i + 1] * np.roll(c, i, axis=-1)
    return out


def circular_convolution_fft(a: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Circular convolution through the DFT: F^{-1}(F(a) o F(c)) (Eq. (2))."""
    b = a.shape[-1]
    return np.fft.irfft(np.fft.rfft(a, axis=-1) * np.fft.rfft(c, axis=-1), n=b, axis=-1)


def sketch_rank1(u, v, w, h, xi, b) -> np.ndarray:
    """Sketch of u (x) v (x) w by Eq. (2): s_{1,u} * s_{2,v} * s_{3,w} (direct)."""
    s1 = count_sketch(u, h[0], xi[0], b)
    s2 = count_sketch(v, h[1], xi[1], b)
    s3 = count_sketch(w, h[2], xi[2], b)
    return circular_convolution(circular_convolution(s1, s2), s3)


def sketch_rank1_fft(u, v, w, h, xi, b) -> np.ndarray:
    """Eq. (2) evaluated with FFTs: F^{-1}(F(s1 u) o F(s2 v) o F(s3 w))."""
    S1 = np.fft.rfft(count_sketch(u, h[0], xi[0], b), axis=-1)
    S2 = np.fft.rfft(count_sketch(v, h[1], xi[1], b), axis=-1)
    S3 = np.fft.rfft(count_sketch(w, h[2], xi[2], b), axis=-1)
    return np.fft.irfft(S1 * S2 * S3, n=b, axis=-1)


def sketch_factors(lam: np.ndarray, A: np.ndarray, h, xi, b) -> np.ndarray:
    """Sketch of sum_r lam_r a_r^{(x)3} by linearity of the sketch (Section 3.1)
    and Eq. (2) per term."""
    s = np.zeros(b, dtype=np.float64)
    for r in range(len(lam)):
        s += float(lam[r]) * sketch_rank1_fft(A[r], A[r], A[r], h, xi, b)
    return s
