"""Colliding-hash symmetric tensor sketches (Section 3.3, Eq. (5)) and the
fast tensor power method on them (Appendix B) -- test infrastructure only.

One hash h: [n] -> [b] and one complex sign sigma(i) = i^q(i), q uniform on
{0, 1, 2, 3} (the 4th roots of unity), per sketch.  The symmetric sketch of a
tensor (Eq. (5)):
    s(t) = sum over (h(i) + h(j) + h(k)) mod b == t of sigma(i) sigma(j) sigma(k) T_ijk,
over all index triples; every permutation of a triple lands in the same bucket
with the same sign, so for a symmetric tensor it equals the sum over
i <= j <= k with multiplicity 6, 3 or 1 (the build the section proposes).

Contractions (Appendix B), <a, c> = sum_t a_t conj(c_t):
  * T(u,u,u) ~ <s, s_X> with the sketch of the upper-triangular part of u^(x)3
        s_X = s_u * s_u * s_u / 6 + s_2 * s_u / 2 + s_3 / 3,
    s_u(t) = sum_{h(i)=t} sigma_i u_i, s_2(t) = sum_{2h(i)=t} sigma_i^2 u_i^2,
    s_3(t) = sum_{3h(i)=t} sigma_i^3 u_i^3 (positions mod b);
  * T(I,u,u)_i ~ <s, s_{Z_i}> / 3, Z_i the symmetrisation of e_i (x) u (x) u,
        s_{Z_i} = s_u * s_u * s_{e_i} / 2 + s_2 * s_{e_i} / 2 + s_{2,e_i u} * s_u + s_{3,e_i u u},
    read off as
        v_i = (1/3) [ conj(sigma_i) (c_1 + c_2)[h(i)] / 2 + conj(sigma_i^2) u_i c_3[2h(i)]
                      + conj(sigma_i^3) u_i^2 s[3h(i)] ],
    c_1 = F^-1(F(s) conj F(s_u)^2), c_2 = F^-1(F(s) conj F(s_2)), c_3 = F^-1(F(s) conj F(s_u)).
    Reading: the printed read-off carries the 1/3 of the footnote on the two
    middle terms only (coefficients 1, 1/6, 1/6, 1); the factor belongs to all
    four -- the printed form is biased, the corrected one unbiased (pinned by
    enumerating every sign draw).
  * The power step takes the median over sketches of Re(v_i), as Algorithm 1.
  * Deflation subtracts lam_hat times the full symmetric sketch of
    u_hat^(x)3, which is s_u * s_u * s_u.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .contract import median


def sigma(q: np.ndarray) -> np.ndarray:
    return np.array([1, 1j, -1, -1j])[np.asarray(q, dtype=np.int64) % 4]


def sym_sketch_dense(T: np.ndarray, h, q, b: int) -> np.ndarray:
    """Eq. (5) over all n^3 entries, by an explicit scatter."""
    T = np.asarray(T, dtype=np.float64)
    n = T.shape[0]
    h = np.asarray(h, dtype=np.int64)
    sg = sigma(q)
    I, J, K = np.indices((n, n, n))
    s = np.zeros(b, dtype=np.complex128)
    np.add.at(s, ((h[I] + h[J] + h[K]) % b).ravel(), (sg[I] * sg[J] * sg[K] * T).ravel())
    return s


def sym_sketch_upper(T: np.ndarray, h, q, b: int) -> np.ndarray:
    """The same sketch from the entries with i <= j <= k only, each weighted by
    the number of distinct permutations of its index triple."""
    T = np.asarray(T, dtype=np.float64)
    n = T.shape[0]
    h = np.asarray(h, dtype=np.int64)
    sg = sigma(q)
    s = np.zeros(b, dtype=np.complex128)
    for i in range(n):
        for j in range(i, n):
            for k in range(j, n):
                mult = 1 if i == j == k else (3 if (i == j or j == k) else 6)
                s[(h[i] + h[j] + h[k]) % b] += mult * sg[i] * sg[j] * sg[k] * T[i, j, k]
    return s


def sym_count_sketch(x: np.ndarray, h, q, b: int, p: int = 1) -> np.ndarray:
    """s_p(t) = sum_{p h(i) = t mod b} sigma_i^p x_i for x [..., n]."""
    x = np.asarray(x)
    h = np.asarray(h, dtype=np.int64)
    w = sigma(q) ** p
    out = np.zeros(x.shape[:-1] + (b,), dtype=np.complex128)
    pos = (p * h) % b
    for i in range(x.shape[-1]):
        out[..., pos[i]] += w[i] * x[..., i]
    return out


def cconv(a: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Circular convolution of complex sequences (FFT route)."""
    return np.fft.ifft(np.fft.fft(a, axis=-1) * np.fft.fft(c, axis=-1), axis=-1)


def cconv_direct(a: np.ndarray, c: np.ndarray) -> np.ndarray:
    b = a.shape[-1]
    out = np.zeros(b, dtype=np.complex128)
    for t in range(b):
        for r in range(b):
            out[(t + r) % b] += a[t] * c[r]
    return out


def sym_tuuu(s: np.ndarray, h, q, u: np.ndarray) -> complex:
    """T(u,u,u) estimate <s, s_X> (real part is the estimate)."""
    b = s.shape[-1]
    s1 = sym_count_sketch(u, h, q, b, 1)
    s2 = sym_count_sketch(u ** 2, h, q, b, 2)
    s3 = sym_count_sketch(u ** 3, h, q, b, 3)
    sX = cconv(cconv(s1, s1), s1) / 6 + cconv(s2, s1) / 2 + s3 / 3
    return complex(np.sum(s * np.conj(sX)))


def sym_tiuu(s: np.ndarray, h, q, u: np.ndarray, coef=(1 / 3, 1 / 6, 1 / 6, 1 / 3)) -> np.ndarray:
    """T(I,u,u) estimate (complex; the real part is the estimate) by the
    read-off above; `coef` are the weights of the terms read at
    (h, h, 2h, 3h); the printed weights are (1, 1/6, 1/6, 1)."""
    b = s.shape[-1]
    h64 = np.asarray(h, dtype=np.int64)
    sg = sigma(q)
    F = np.fft.fft(s)
    U1 = np.fft.fft(sym_count_sketch(u, h, q, b, 1))
    U2 = np.fft.fft(sym_count_sketch(u ** 2, h, q, b, 2))
    c1 = np.fft.ifft(F * np.conj(U1) ** 2)
    c2 = np.fft.ifft(F * np.conj(U2))
    c3 = np.fft.ifft(F * np.conj(U1))
    a, bb, c, d = coef
    # coef[1] multiplies c_1 and coef[2] c_2 (both read at h); coef[0] the
    # 2h term and coef[3] the 3h term, in the order of the printed equation.
    return (bb * np.conj(sg) * c1[h64] + c * np.conj(sg) * c2[h64]
            + a * np.conj(sg ** 2) * u * c3[(2 * h64) % b]
            + d * np.conj(sg ** 3) * u ** 2 * s[(3 * h64) % b])


def sym_tiuu_direct(s: np.ndarray, h, q, u: np.ndarray) -> np.ndarray:
    """<s, s_{Z_i}> / 3 with s_{Z_i} formed by direct convolutions (no FFT)."""
    b = s.shape[-1]
    n = u.shape[-1]
    s1 = sym_count_sketch(u, h, q, b, 1)
    s2 = sym_count_sketch(u ** 2, h, q, b, 2)
    s11 = cconv_direct(s1, s1)
    v = np.zeros(n, dtype=np.complex128)
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        se = sym_count_sketch(e, h, q, b, 1)
        s2e = sym_count_sketch(e * u, h, q, b, 2)
        s3e = sym_count_sketch(e * u * u, h, q, b, 3)
        sZ = (cconv_direct(s11, se) / 2 + cconv_direct(s2, se) / 2 + cconv_direct(s2e, s1) + s3e)
        v[i] = np.sum(s * np.conj(sZ)) / 3
    return v


def sym_power_update(S: np.ndarray, h, q, U: np.ndarray):
    """One power step on symmetric sketches S [B][b] (complex, time domain):
    V[tau][m] = Re T(I,u,u) estimates, vbar = median over m, u <- vbar/||vbar||
    (kept and flagged when the norm is zero or not finite)."""
    B = S.shape[0]
    L = U.shape[0]
    V = np.zeros((L, B, U.shape[1]))
    for tau in range(L):
        for m in range(B):
            V[tau, m] = np.real(sym_tiuu(S[m], h[m], q[m], U[tau]))
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


@dataclasses.dataclass
class SymResult:
    lam: np.ndarray
    U: np.ndarray
    tau: np.ndarray
    flags: np.ndarray
    S: np.ndarray
    lam_tau: np.ndarray = None   # [k][L] selection values of each component's restarts


def rtpm_symmetric(S: np.ndarray, h, q, k: int, L: int, T: int, u0: np.ndarray) -> SymResult:
    """Algorithm 1 on symmetric sketches: T power steps per restart, selection
    by the median over sketches of Re T(u,u,u) (lowest restart on ties, a
    non-finite value never wins), lambda_hat at the renormalised winner, and
    deflation of every sketch by lambda_hat (s_u * s_u * s_u)."""
    S = np.array(S, dtype=np.complex128, copy=True)
    B, b = S.shape
    n = u0.shape[-1]
    lam_out, U_out = np.zeros(k), np.zeros((k, n))
    tau_out = np.zeros(k, dtype=np.int64)
    flags = np.zeros((k, L), dtype=np.int32)
    lam_tau_out = np.zeros((k, L))
    for c in range(k):
        U = np.array(u0[c], dtype=np.float64, copy=True)
        for _ in range(T):
            _, U, f = sym_power_update(S, h, q, U)
            flags[c] |= f
        lam_tau = np.array([median(np.array([np.real(sym_tuuu(S[m], h[m], q[m], U[tau])) for m in range(B)]),
                                   axis=0) for tau in range(L)])
        key = np.where(np.isfinite(lam_tau), lam_tau, -np.inf)
        tau = int(np.argmax(key))
        u_hat = U[tau] / np.linalg.norm(U[tau])
        lam_hat = float(median(np.array([np.real(sym_tuuu(S[m], h[m], q[m], u_hat)) for m in range(B)]),
                               axis=0))
        for m in range(B):
            s1 = sym_count_sketch(u_hat, h[m], q[m], b, 1)
            S[m] -= lam_hat * cconv(cconv(s1, s1), s1)
        lam_out[c], U_out[c], tau_out[c] = lam_hat, u_hat, tau
        lam_tau_out[c] = lam_tau
    return SymResult(lam=lam_out, U=U_out, tau=tau_out, flags=flags, S=S, lam_tau=lam_tau_out)
