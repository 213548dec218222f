"""Pins for the oracle's whitened LDA moment (Appendix D), against what the
mathematics fixes:

  * the per-document third and second moment estimates against brute force
    over all ordered triples / pairs of distinct word positions;
  * Eq. (td) against the whitened third-moment estimate N_d(W, W, W);
  * the moment combination of Eq. (moment2)/(moment3) applied to the exact
    population moments of an LDA model against the closed forms
    sum_i alpha_i mu_i mu_i^T / (alpha0 (alpha0+1)) and
    2 sum_i alpha_i mu_i^(x)3 / (alpha0 (alpha0+1)(alpha0+2));
  * the whitened per-document route against contracting the explicit V^3
    moment with W on every mode.
"""
import numpy as np
import pytest

from oracle import lda
from paper_1506_04448_amd.workloads import lda_corpus


def _counts(words, V):
    n = np.zeros(V)
    for w in words:
        n[w] += 1
    return n


@pytest.mark.parametrize("words", [[0, 1, 1, 2, 2, 2, 4], [3, 3, 3], [0, 1, 2, 3, 4, 0, 0, 1]])
def test_document_moments_equal_bruteforce(words):
    V = max(words) + 1
    n = _counts(words, V)
    np.testing.assert_allclose(lda.doc_third_moment(n), lda.doc_third_moment_bruteforce(words),
                               atol=1e-15)
    np.testing.assert_allclose(lda.doc_second_moment(n), lda.doc_second_moment_bruteforce(words),
                               atol=1e-15)


def test_eq_td_equals_whitened_doc_moment():
    rng = np.random.default_rng(1)
    V, K = 9, 4
    W = rng.standard_normal((V, K))
    n = rng.integers(0, 4, V).astype(float)
    n[0] = 3
    Nd = lda.doc_third_moment(n)
    np.testing.assert_allclose(lda.whitened_doc_term(n, W), np.einsum("ijk,ia,jb,kc->abc", Nd, W, W, W),
                               atol=1e-12)


def test_combination_matches_population_closed_forms():
    rng = np.random.default_rng(2)
    V, K = 7, 3
    Phi = rng.dirichlet(np.ones(V), size=K).T
    alpha = rng.uniform(0.2, 2.0, K)
    a0 = alpha.sum()
    M1, E2, E3 = lda.population_moments(Phi, alpha)
    M2 = lda.combine_m2(E2, M1, a0)
    M3 = lda.combine_m3(E3, E2, M1, a0)
    np.testing.assert_allclose(M2, (Phi * alpha) @ Phi.T / (a0 * (a0 + 1)), atol=1e-14)
    M3_ref = 2.0 * np.einsum("r,ir,jr,kr->ijk", alpha, Phi, Phi, Phi) / (a0 * (a0 + 1) * (a0 + 2))
    np.testing.assert_allclose(M3, M3_ref, atol=1e-14)
    # population moments are a valid probability model: M1 sums to one
    assert M1.sum() == pytest.approx(1.0)
    assert E3.sum() == pytest.approx(1.0)


def test_whitened_route_equals_explicit_route():
    C = lda_corpus(D=40, V=12, K=3, seed=4, mean_len=6.0, min_len=1)
    rng = np.random.default_rng(5)
    W = rng.standard_normal((C.V, 3))
    a0 = 1.7
    explicit = lda.explicit_m3(C, a0)
    np.testing.assert_allclose(lda.whitened_m3(C, W, a0),
                               np.einsum("ijk,ia,jb,kc->abc", explicit, W, W, W), atol=1e-12)
    # short documents (m < 3) are dropped, not counted
    lens = np.diff(C.rowptr)
    m = np.array([C.cnt[C.rowptr[d]:C.rowptr[d + 1]].sum() for d in range(len(lens))])
    assert (m < 3).any()
