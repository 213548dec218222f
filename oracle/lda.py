"""Whitened third-order LDA moment and its sketch (oracle side) -- test
infrastructure only.

Spectral LDA (Appendix D) decomposes the whitened third moment
  M3 = E[x1 (x) x2 (x) x3] - a (E[x1 (x) x2 (x) M1] + E[x1 (x) M1 (x) x2] + E[M1 (x) x1 (x) x2])
       + c M1 (x) M1 (x) M1,        a = alpha0 / (alpha0 + 2),
                                    c = 2 alpha0^2 / ((alpha0 + 1)(alpha0 + 2)),
contracted with a whitening matrix W (V x K) on every mode.  The word
moments are estimated per document from its counts n (length m) without
replacement: the third moment by N_d of Appendix D (its all-equal case is
n_i (n_i - 1)(n_i - 2); the printed n_i (n_j - 1)(n_k - 2) with i = j = k is
the same thing), the second by (n n^T - diag n) / (m (m - 1)), and the
document estimates are averaged over the documents; documents with fewer than
three words are dropped.  The whitened document term follows Eq. (td) of
Appendix D with p = W^T n and w_i the i-th row of W.  The paper writes
p = W n and, for the cross term, sum_i n_i p (x) p (x) q; the readings here
are p = W^T n and the document's whitened second moment
(p p^T - sum_i n_i w_i w_i^T) / (m (m - 1)) times q = W^T M1.

Pinned by tests/test_oracle_lda_pins.py: the moment formulas against brute
force over ordered triples / pairs of distinct word positions, Eq. (td)
against the whitened N_d, the combination against the closed forms of the
population moments (sum_i alpha_i mu_i^(x)3 / (alpha0 (alpha0 + 1)(alpha0 + 2))
up to the factor 2), and the whitened route against the explicit V^3 route.
"""
from __future__ import annotations

import itertools

import numpy as np

from .sketch import sketch_dense


def _coefs(alpha0: float):
    a = alpha0 / (alpha0 + 2.0)
    c = 2.0 * alpha0 ** 2 / ((alpha0 + 1.0) * (alpha0 + 2.0))
    return a, c


def doc_third_moment(n: np.ndarray) -> np.ndarray:
    """N_d: the unbiased estimate of E[x1 (x) x2 (x) x3] from one document's
    counts (V^3; small V only)."""
    n = np.asarray(n, dtype=np.float64)
    m = n.sum()
    N = np.einsum("i,j,k->ijk", n, n, n)
    V = n.size
    idx = np.arange(V)
    # i = j (and k free), j = k, i = k corrections, then the all-equal case
    N[idx, idx, :] -= np.outer(n, n)
    N[:, idx, idx] -= np.outer(n, n)
    N[idx, :, idx] -= np.outer(n, n)
    N[idx, idx, idx] += 2.0 * n
    return N / (m * (m - 1.0) * (m - 2.0))


def doc_third_moment_bruteforce(words) -> np.ndarray:
    """Average of e_a (x) e_b (x) e_c over all ordered triples of distinct
    word positions of the document (words: list of word ids)."""
    V = int(max(words)) + 1
    out = np.zeros((V, V, V))
    cnt = 0
    for a, b, c in itertools.permutations(range(len(words)), 3):
        out[words[a], words[b], words[c]] += 1.0
        cnt += 1
    return out / cnt


def doc_second_moment(n: np.ndarray) -> np.ndarray:
    n = np.asarray(n, dtype=np.float64)
    m = n.sum()
    return (np.outer(n, n) - np.diag(n)) / (m * (m - 1.0))


def doc_second_moment_bruteforce(words) -> np.ndarray:
    V = int(max(words)) + 1
    out = np.zeros((V, V))
    cnt = 0
    for a, b in itertools.permutations(range(len(words)), 2):
        out[words[a], words[b]] += 1.0
        cnt += 1
    return out / cnt


def whitened_doc_term(n: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Eq. (td) divided by m (m-1)(m-2):
    (p^(x)3 - sum_i n_i (w_i w_i p + w_i p w_i + p w_i w_i) + 2 sum_i n_i w_i^(x)3) / (m(m-1)(m-2))."""
    n = np.asarray(n, dtype=np.float64)
    m = n.sum()
    p = W.T @ n
    T = np.einsum("i,j,k->ijk", p, p, p)
    for i in np.flatnonzero(n):
        w = W[i]
        T -= n[i] * (np.einsum("i,j,k->ijk", w, w, p) + np.einsum("i,j,k->ijk", w, p, w)
                     + np.einsum("i,j,k->ijk", p, w, w))
        T += 2.0 * n[i] * np.einsum("i,j,k->ijk", w, w, w)
    return T / (m * (m - 1.0) * (m - 2.0))


def combine_m3(E3: np.ndarray, E2: np.ndarray, M1: np.ndarray, alpha0: float) -> np.ndarray:
    """The combination of Eq. (moment3) from E[x1 x2 x3], E[x1 x2] and M1
    (the cross terms E[x1 (x) x2 (x) M1] and its permutations are E2 (x) M1)."""
    a, c = _coefs(alpha0)
    cross = (np.einsum("ij,k->ijk", E2, M1) + np.einsum("ik,j->ijk", E2, M1)
             + np.einsum("jk,i->ijk", E2, M1))
    return E3 - a * cross + c * np.einsum("i,j,k->ijk", M1, M1, M1)


def combine_m2(E2: np.ndarray, M1: np.ndarray, alpha0: float) -> np.ndarray:
    return E2 - alpha0 / (alpha0 + 1.0) * np.outer(M1, M1)


def population_moments(Phi: np.ndarray, alpha: np.ndarray):
    """Exact word moments of the LDA model (Dirichlet moments of the topic
    mixture pushed through Phi): (M1, E[x1 x2], E[x1 x2 x3])."""
    a0 = float(np.sum(alpha))
    Eh = alpha / a0
    Ehh = (np.outer(alpha, alpha) + np.diag(alpha)) / (a0 * (a0 + 1.0))
    K = alpha.size
    Ehhh = np.einsum("i,j,k->ijk", alpha, alpha, alpha)
    idx = np.arange(K)
    Ehhh[idx, idx, :] += np.outer(alpha, alpha)
    Ehhh[idx, :, idx] += np.outer(alpha, alpha)
    Ehhh[:, idx, idx] += np.outer(alpha, alpha)
    Ehhh[idx, idx, idx] += 2.0 * alpha
    Ehhh /= a0 * (a0 + 1.0) * (a0 + 2.0)
    M1 = Phi @ Eh
    E2 = Phi @ Ehh @ Phi.T
    E3 = np.einsum("abc,ia,jb,kc->ijk", Ehhh, Phi, Phi, Phi)
    return M1, E2, E3


def _docs(corpus):
    """(counts vector, length) of every document with at least three words."""
    V = corpus.V
    for d in range(len(corpus.rowptr) - 1):
        lo, hi = corpus.rowptr[d], corpus.rowptr[d + 1]
        m = float(np.sum(corpus.cnt[lo:hi]))
        if m < 3:
            continue
        n = np.zeros(V)
        n[corpus.col[lo:hi]] = corpus.cnt[lo:hi]
        yield n, m


def empirical_m1(corpus) -> np.ndarray:
    docs = list(_docs(corpus))
    return np.mean([n / m for n, m in docs], axis=0)


def whitened_m3(corpus, W: np.ndarray, alpha0: float) -> np.ndarray:
    """M3(W, W, W) from the per-document whitened terms (K^3, FP64)."""
    a, c = _coefs(alpha0)
    docs = list(_docs(corpus))
    D = len(docs)
    q = W.T @ np.mean([n / m for n, m in docs], axis=0)
    K = W.shape[1]
    T = np.zeros((K, K, K))
    for n, m in docs:
        T += whitened_doc_term(n, W)
        p = W.T @ n
        E2w = (np.outer(p, p) - (W.T * n) @ W) / (m * (m - 1.0))
        T -= a * (np.einsum("ij,k->ijk", E2w, q) + np.einsum("ik,j->ijk", E2w, q)
                  + np.einsum("jk,i->ijk", E2w, q))
    T /= D
    return T + c * np.einsum("i,j,k->ijk", q, q, q)


def explicit_m3(corpus, alpha0: float) -> np.ndarray:
    """M3 over the V^3 word space from the averaged document estimates (small V)."""
    docs = list(_docs(corpus))
    E3 = np.mean([doc_third_moment(n) for n, _ in docs], axis=0)
    E2 = np.mean([doc_second_moment(n) for n, _ in docs], axis=0)
    M1 = np.mean([n / m for n, m in docs], axis=0)
    return combine_m3(E3, E2, M1, alpha0)


def sketch_docs(corpus, W: np.ndarray, alpha0: float, h, xi, b: int) -> np.ndarray:
    """The B sketches of M3(W, W, W) by Eq. (1) over the explicit K^3 tensor."""
    T = whitened_m3(corpus, W, alpha0)
    return np.stack([sketch_dense(T, h[m], xi[m], b) for m in range(h.shape[0])])


# ---- Fast spectral LDA (Appendix D, Algorithm 3): whitening and recovery ----

def empirical_m2(corpus, alpha0: float) -> np.ndarray:
    """M2 of Eq. (moment2) from the averaged document estimates (V x V)."""
    docs = list(_docs(corpus))
    E2 = np.mean([doc_second_moment(n) for n, _ in docs], axis=0)
    M1 = np.mean([n / m for n, m in docs], axis=0)
    return combine_m2(E2, M1, alpha0)


def whitening_exact(M2: np.ndarray, K: int):
    """W = U_K diag(1/sqrt(sigma_K)) from the K largest-magnitude eigenpairs of
    the symmetric M2 (its truncated SVD); returns (W, sigma)."""
    d, E = np.linalg.eigh(M2)
    order = np.argsort(-np.abs(d), kind="stable")[:K]
    sig = np.abs(d[order])
    return E[:, order] / np.sqrt(sig), sig


def orth_gram(Y: np.ndarray, rel: float = 1e-12) -> np.ndarray:
    """Orthonormal basis of range(Y) through the eigenpairs of Y^T Y:
    Q = Y E diag(1/sqrt(d)) (columns with d <= rel max d dropped to zero)."""
    d, E = np.linalg.eigh(Y.T @ Y)
    keep = d > rel * d.max()
    Q = np.zeros_like(Y)
    Q[:, keep] = (Y @ E[:, keep]) / np.sqrt(d[keep])
    return Q


def whitening_subspace(M2: np.ndarray, Omega: np.ndarray, iters: int):
    """The randomized truncated SVD the library runs: Y = M2 Omega; `iters`
    rounds of Q = orth(Y), Y = M2 Q; then Q = orth(Y), B = Q^T M2 Q and
    W = Q E_B diag(1/sqrt|d_B|) over B's eigenpairs by decreasing |d|."""
    Y = M2 @ Omega
    for _ in range(iters):
        Y = M2 @ orth_gram(Y)
    Q = orth_gram(Y)
    Bm = Q.T @ (M2 @ Q)
    Bm = (Bm + Bm.T) / 2
    d, E = np.linalg.eigh(Bm)
    order = np.argsort(-np.abs(d), kind="stable")
    sig = np.abs(d[order])
    return (Q @ E[:, order]) / np.sqrt(sig), sig


def recover(lam: np.ndarray, V: np.ndarray, W: np.ndarray, alpha0: float):
    """Algorithm 3's output: alpha_i = 4 alpha0 (alpha0 + 1) / ((alpha0 + 2)^2 lam_i^2)
    and mu_i = (alpha0 + 2)/2 lam_i (W^+)^T v_i; V [k][K] rows, W [V][K]."""
    alpha = 4.0 * alpha0 * (alpha0 + 1.0) / ((alpha0 + 2.0) ** 2 * lam ** 2)
    mu = (alpha0 + 2.0) / 2.0 * lam[:, None] * (np.linalg.pinv(W).T @ V.T).T
    return alpha, mu
