"""Seeded synthetic inputs shaped like the paper's workloads.

This module builds inputs only: planted symmetric tensors, rank-1 factor
lists, start vectors drawn by numpy, and a synthetic LDA-shaped corpus.  It
holds none of the sketching or power-method arithmetic, so both the HIP path
and the CPU oracle can take their inputs from here.

Construction of the planted tensors follows the synthetic setting of the
paper's experiments (Section 5.1): an orthonormal basis, positive weights and
a symmetric Gaussian noise tensor drawn for i<=j<=k and copied to every
permutation of the indices.  The noise standard deviation is 1/n^1.5 times
the noise level, so that the Frobenius norm of the noise is about the level.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Planted:
    T: np.ndarray          # [n][n][n] row-major, float64 or float32
    lam: np.ndarray        # [k] float64 planted weights
    V: np.ndarray          # [k][n] float64 planted unit vectors (rows)
    noise: float


def symmetric_noise(rng: np.random.Generator, n: int) -> np.ndarray:
    """Symmetric Gaussian tensor with std 1/n^1.5 per entry.

    Entries with i<=j<=k are drawn independently; every other entry copies
    the entry at its sorted index triple (Section 5.1 of the paper).
    """
    G = rng.standard_normal((n, n, n)) * (1.0 / n ** 1.5)
    idx = np.indices((n, n, n), dtype=np.int32).reshape(3, -1)
    idx.sort(axis=0)
    E = G[idx[0], idx[1], idx[2]].reshape(n, n, n)
    return E


def planted_tensor(n: int, k: int, noise: float, seed: int,
                   lam_range=(1.0, 2.0), dtype=np.float64) -> Planted:
    """T = sum_i lam_i v_i^{(x)3} + noise * E with v_i orthonormal (QR of a
    Gaussian n x k matrix) and lam_i ~ U[lam_range]."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    lam = rng.uniform(lam_range[0], lam_range[1], size=k)
    T = np.einsum("r,ir,jr,kr->ijk", lam, Q, Q, Q, optimize=True)
    if noise != 0.0:
        T = T + noise * symmetric_noise(rng, n)
    return Planted(T=np.ascontiguousarray(T.astype(dtype)), lam=lam,
                   V=np.ascontiguousarray(Q.T), noise=noise)


def random_unit_vectors(rng: np.random.Generator, rows: int, n: int) -> np.ndarray:
    X = rng.standard_normal((rows, n))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    return X


def start_vectors(seed: int, k: int, L: int, n: int) -> np.ndarray:
    """Start vectors u0[k][L][n], each uniform on the unit sphere."""
    rng = np.random.default_rng(seed)
    return random_unit_vectors(rng, k * L, n).reshape(k, L, n)


@dataclasses.dataclass
class FactorInstance:
    n: int
    k: int
    b: int
    lam: np.ndarray        # [k] float64
    A: np.ndarray          # [k][n] float64, unit rows (not orthogonal)


def factor_instances(count: int, seed: int, n_range=(100, 2000), k_range=(5, 50),
                     lam_range=(1.0, 10.0), b_choices=(4096, 16384, 65536)):
    """Uneven low-rank tensors given only by their factors."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        b = int(rng.choice(np.asarray(b_choices)))
        lam = rng.uniform(lam_range[0], lam_range[1], size=k)
        A = random_unit_vectors(rng, k, n)
        out.append(FactorInstance(n=n, k=k, b=b, lam=lam, A=A))
    return out


@dataclasses.dataclass
class Corpus:
    rowptr: np.ndarray     # [D+1] int32
    col: np.ndarray        # [nnz] int32 word ids
    cnt: np.ndarray        # [nnz] int32 counts
    V: int
    K: int
    alpha: np.ndarray      # [K]
    Phi: np.ndarray        # [V][K] topic-word distributions (columns sum to 1)


def lda_corpus(D: int, V: int, K: int, seed: int, mean_len: float = 150.0,
               beta: float = 0.01, alpha: float = 0.1, min_len: int = 3) -> Corpus:
    """Synthetic LDA corpus: Phi_k ~ Dir(beta 1_V), theta_d ~ Dir(alpha 1_K),
    m_d ~ Poisson(mean_len) (resampled below min_len), words ~ Cat(Phi theta_d).
    Word counts are stored as CSR with sorted word ids."""
    rng = np.random.default_rng(seed)
    Phi = rng.dirichlet(np.full(V, beta), size=K).T.copy()      # [V][K]
    alph = np.full(K, alpha)
    rowptr = np.zeros(D + 1, dtype=np.int64)
    cols, cnts = [], []
    for d in range(D):
        m = 0
        while m < min_len:
            m = int(rng.poisson(mean_len))
        theta = rng.dirichlet(alph)
        p = Phi @ theta
        p /= p.sum()
        c = rng.multinomial(m, p)
        nz = np.flatnonzero(c)
        cols.append(nz.astype(np.int32))
        cnts.append(c[nz].astype(np.int32))
        rowptr[d + 1] = rowptr[d] + nz.size
    return Corpus(rowptr=rowptr.astype(np.int32), col=np.concatenate(cols),
                  cnt=np.concatenate(cnts), V=V, K=K, alpha=alph, Phi=Phi)


def lda_corpus_fast(D: int, V: int, K: int, seed: int, mean_len: float = 150.0,
                    beta: float = 0.01, alpha: float = 0.1, min_len: int = 3,
                    batch: int = 50000) -> Corpus:
    """The same generative model as lda_corpus, drawn in bulk for large D:
    per-document topic counts ~ Multinomial(m_d, theta_d), then each topic's
    words ~ Cat(Phi_k) by inverse-CDF sampling, merged into CSR counts.  (Its
    random stream differs from lda_corpus's.)"""
    rng = np.random.default_rng(seed)
    Phi = rng.dirichlet(np.full(V, beta), size=K).T.copy()      # [V][K]
    cdf = np.cumsum(Phi, axis=0)
    cdf /= cdf[-1]
    alph = np.full(K, alpha)
    rows, cols, cnts = [np.zeros(1, dtype=np.int64)], [], []
    total = 0
    for d0 in range(0, D, batch):
        nd = min(batch, D - d0)
        m = rng.poisson(mean_len, size=nd)
        while (m < min_len).any():
            bad = m < min_len
            m[bad] = rng.poisson(mean_len, size=int(bad.sum()))
        theta = rng.dirichlet(alph, size=nd)
        zc = rng.multinomial(m, theta)                             # [nd][K] topic counts
        doc_of = np.repeat(np.arange(nd), m)
        words = np.empty(int(m.sum()), dtype=np.int64)
        # positions grouped by topic: for each document, its words of topic k
        topic = np.repeat(np.tile(np.arange(K), nd), zc.ravel())
        for k in range(K):
            sel = np.flatnonzero(topic == k)
            if sel.size:
                words[sel] = np.searchsorted(cdf[:, k], rng.random(sel.size), side="right")
        np.minimum(words, V - 1, out=words)
        key = np.unique(doc_of * V + words, return_counts=True)
        d_idx, w_idx = np.divmod(key[0], V)
        per_doc = np.bincount(d_idx, minlength=nd)
        rows.append(total + np.cumsum(per_doc))
        total += int(per_doc.sum())
        cols.append(w_idx.astype(np.int32))
        cnts.append(key[1].astype(np.int32))
    rowptr = np.concatenate(rows)
    return Corpus(rowptr=rowptr.astype(np.int32), col=np.concatenate(cols),
                  cnt=np.concatenate(cnts), V=V, K=K, alpha=alph, Phi=Phi)


def population_whitening(Phi: np.ndarray, alpha: np.ndarray) -> np.ndarray:
    """W (V x K) with W^T M2 W = I for the population second moment
    M2 = sum_i alpha_i mu_i mu_i^T / (alpha0 (alpha0 + 1)) of the LDA model."""
    a0 = float(np.sum(alpha))
    A = Phi * np.sqrt(alpha / (a0 * (a0 + 1.0)))
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    return U / s


@dataclasses.dataclass
class FullRankTensor:
    T: object              # torch float32 [n][n][n] on the requested device
    lam: np.ndarray        # [n] float64 weights after normalisation (descending)
    V: np.ndarray          # [n][n] float64 orthonormal basis (rows)
    sigma: float


def full_rank_tensor(n: int, sigma: float, seed: int, device="cpu", chunk: int = 50) -> FullRankTensor:
    """The synthetic tensors of the paper's accuracy table (Section 5.1,
    Table 5): T = normalize(sum_{i<=n} lam_i v_i^{(x)3}) + E with a random
    orthonormal basis {v_i} (QR of a seeded Gaussian n x n matrix), lam_i = 1/i
    before normalisation, the signal scaled to unit Frobenius norm (exact:
    ||sum lam_i v_i^{(x)3}||_F^2 = sum lam_i^2 for an orthonormal basis), and a
    symmetric Gaussian E drawn for i<=j<=k and copied to every permutation of
    the indices, with variance sigma/n^3 per entry so that E||E||_F^2 = sigma.

    Built with torch on `device` (the n = 1000 tensor takes 4 GB in FP32): the
    signal slab by slab as an FP64 matrix product, the noise from a seeded
    torch generator on that device, gathered at the sorted index triples.
    """
    import torch
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 1.0 / np.arange(1, n + 1, dtype=np.float64)
    lam /= np.linalg.norm(lam)
    T = _device_symmetric_tensor(Q, lam, float(np.sqrt(sigma / float(n) ** 3)), seed, device, chunk)
    return FullRankTensor(T=T, lam=lam, V=np.ascontiguousarray(Q.T), sigma=sigma)


def _device_symmetric_tensor(Q: np.ndarray, lam: np.ndarray, noise_std: float, seed: int, device,
                             chunk: int):
    """FP32 [n][n][n] tensor sum_r lam_r q_r^{(x)3} + E on `device`, with E
    symmetric Gaussian of standard deviation `noise_std` per entry: drawn
    once per sorted index triple (a seeded torch generator on the device) and
    gathered at every permutation.  The signal is formed slab by slab as an
    FP64 matrix product."""
    import torch
    n = Q.shape[0]
    dev = torch.device(device)
    Qd = torch.from_numpy(Q).to(dev)
    QlT = (Qd * torch.from_numpy(lam).to(dev)).T.contiguous()   # [r][k]: lam_r q_k,r
    T = torch.empty((n, n, n), dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    G = torch.randn((n, n, n), generator=gen, dtype=torch.float32, device=dev)
    G.mul_(noise_std)
    Gf = G.view(-1)
    jj = torch.arange(n, device=dev).view(n, 1).expand(n, n)
    kk = torch.arange(n, device=dev).view(1, n).expand(n, n)
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        # signal: T[i, j, k] = sum_r q_ir q_jr lam_r q_kr
        A = (Qd[i0:i1, None, :] * Qd[None, :, :]).reshape((i1 - i0) * n, Q.shape[1])
        T[i0:i1] = (A @ QlT).view(i1 - i0, n, n).to(torch.float32)
        # noise: E[i, j, k] = G[sorted(i, j, k)]
        ii = torch.arange(i0, i1, device=dev).view(-1, 1, 1).expand(i1 - i0, n, n)
        j = jj.unsqueeze(0).expand(i1 - i0, n, n)
        k = kk.unsqueeze(0).expand(i1 - i0, n, n)
        lo = torch.minimum(torch.minimum(ii, j), k)
        hi = torch.maximum(torch.maximum(ii, j), k)
        mid = ii + j + k - lo - hi
        T[i0:i1] += Gf[(lo * n + mid) * n + hi]
    del G, Gf
    return T


def planted_tensor_device(n: int, k: int, noise: float, seed: int, device="cpu", chunk: int = 50,
                          lam_range=(1.0, 2.0)):
    """The planted construction of `planted_tensor` (orthonormal v_i from the
    QR of a seeded Gaussian n x k matrix, lam_i ~ U[lam_range], plus noise
    times a symmetric Gaussian E of standard deviation 1/n^1.5 per entry) as
    an FP32 tensor built with torch on `device`: the n = 1000 tensor of the
    differentiation workload takes 4 GB.  Returns a `Planted` whose T is that
    torch tensor."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    lam = rng.uniform(lam_range[0], lam_range[1], size=k)
    T = _device_symmetric_tensor(Q, lam, noise / float(n) ** 1.5, seed, device, chunk)
    return Planted(T=T, lam=lam, V=np.ascontiguousarray(Q.T), noise=noise)


def sym_tables(seed: int, n: int, b: int, B: int):
    """Colliding-hash tables for B sketches: h [B][n] uniform on [0, b) and
    q [B][n] uniform on {0, 1, 2, 3} (the sign is i^q), from numpy."""
    rng = np.random.default_rng(seed)
    h = rng.integers(0, b, size=(B, n), dtype=np.uint32)
    q = rng.integers(0, 4, size=(B, n)).astype(np.uint8)
    return h, q
