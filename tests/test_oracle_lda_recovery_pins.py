"""Pins of the spectral-LDA whitening and recovery (Appendix D, Algorithm 3):

  * from the exact population moments (closed forms of the Dirichlet
    moments), whitening, the orthogonal decomposition of M3(W, W, W) and the
    recovery formulas return the model's alpha and topic vectors exactly;
  * the randomized subspace iteration converges to the exact truncated
    eigendecomposition (W W^T and sigma agree) on an empirical M2, and equals
    it to rounding, with or without power rounds, when M2 has rank exactly K;
  * the orthonormalisation through the Gram eigenpairs gives Q^T Q = I.
"""
import numpy as np

from oracle import lda
from paper_1506_04448_amd.workloads import lda_corpus


def _model(V, K, seed):
    rng = np.random.default_rng(seed)
    Phi = rng.dirichlet(np.full(V, 0.3), size=K).T          # V x K, columns sum to 1
    alpha = rng.uniform(0.2, 1.0, K)
    return Phi, alpha


def test_population_moments_give_back_the_model():
    V, K = 30, 4
    Phi, alpha = _model(V, K, 1)
    a0 = float(alpha.sum())
    M1, E2, E3 = lda.population_moments(Phi, alpha)
    M2 = lda.combine_m2(E2, M1, a0)
    M3 = lda.combine_m3(E3, E2, M1, a0)
    W, sig = lda.whitening_exact(M2, K)
    np.testing.assert_allclose(W.T @ M2 @ W, np.eye(K), atol=1e-10)
    T = np.einsum("abc,ai,bj,ck->ijk", M3, W, W, W)
    # orthogonal decomposition: eigenvectors of T(I, I, theta) for a generic theta
    theta = np.random.default_rng(0).standard_normal(K)
    _, Vv = np.linalg.eigh(np.einsum("ijk,k->ij", T, theta))
    lam = np.einsum("ijk,ir,jr,kr->r", T, Vv, Vv, Vv)
    Vv = Vv * np.sign(lam)
    lam = np.abs(lam)
    alpha_hat, mu_hat = lda.recover(lam, Vv.T, W, a0)
    order = np.argsort(alpha_hat)
    ref = np.argsort(alpha)
    np.testing.assert_allclose(alpha_hat[order], alpha[ref], rtol=1e-8)
    np.testing.assert_allclose(mu_hat[order], Phi.T[ref], atol=1e-9)


def test_subspace_iteration_converges_to_exact_whitening():
    C = lda_corpus(D=400, V=60, K=5, seed=3, mean_len=40.0, min_len=3)
    a0 = float(C.alpha.sum())
    M2 = lda.empirical_m2(C, a0)
    K = 5
    W, sig = lda.whitening_exact(M2, K)
    Om = np.random.default_rng(4).standard_normal((60, K))
    Ws, sigs = lda.whitening_subspace(M2, Om, 40)
    np.testing.assert_allclose(sigs, sig, rtol=1e-8)
    np.testing.assert_allclose(Ws @ Ws.T, W @ W.T, atol=1e-6 * np.abs(W @ W.T).max())


def test_gram_orthonormalisation():
    Y = np.random.default_rng(5).standard_normal((50, 7))
    Q = lda.orth_gram(Y)
    np.testing.assert_allclose(Q.T @ Q, np.eye(7), atol=1e-12)
    np.testing.assert_allclose(Q @ (Q.T @ Y), Y, atol=1e-12)


def test_subspace_whitening_is_exact_when_m2_has_rank_k():
    """With M2 = A diag(s) A^T of rank exactly K (signs mixed, as an empirical
    M2's leading part can be), the range of M2 Omega is range(A) for a generic
    Omega, so even without power rounds the randomized whitening must equal
    the exact one: W^T M2 W = I, the same |eigenvalues| and the same W W^T."""
    rng = np.random.default_rng(11)
    V, K = 40, 6
    A = rng.standard_normal((V, K))
    s = np.array([5.0, -3.0, 2.0, 1.5, -0.7, 0.4])
    M2 = (A * s) @ A.T
    W, sig = lda.whitening_exact(M2, K)
    for iters in (0, 1, 3):
        Om = rng.standard_normal((V, K))
        Ws, sigs = lda.whitening_subspace(M2, Om, iters)
        np.testing.assert_allclose(sigs, sig, rtol=1e-10)
        G = Ws.T @ M2 @ Ws
        np.testing.assert_allclose(np.abs(G), np.eye(K), atol=1e-10)
        np.testing.assert_allclose(Ws @ Ws.T, W @ W.T, atol=1e-10 * np.abs(W @ W.T).max())
