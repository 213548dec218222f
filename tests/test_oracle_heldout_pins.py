"""Pins of the oracle's held-out likelihood (Section 5.2): the simplex-
constrained least-squares fit of a document's mixing vector and its average
log-likelihood.

* brute force: for K <= 7 the active-set result equals the best
  equality-constrained solution over every support (the definition of the
  argmin of a strictly convex programme over the simplex);
* optimality: at K = 100 the result satisfies the KKT conditions (feasible,
  equal gradient on the support, no smaller gradient off it);
* special cases: a document drawn from one column of Phi exactly (w = Phi e_j)
  is fitted by pi = e_j with L_d = sum_i w_i ln Phi[i, j]; a vertex optimum and
  an interior optimum both occur.
A dropped term of the gradient, a wrong sign in the multipliers or a wrong
ratio test moves the result off the brute-force optimum.
"""
import numpy as np
import pytest

from oracle import heldout as H


def _phi(rng, V, K, conc=0.05):
    P = rng.gamma(conc, size=(V, K)) + 1e-12
    return P / P.sum(axis=0, keepdims=True)


@pytest.mark.parametrize("K,V,seed", [(3, 20, 1), (5, 40, 2), (7, 60, 3), (6, 15, 4)])
def test_active_set_equals_bruteforce(K, V, seed):
    rng = np.random.default_rng(seed)
    Phi = _phi(rng, V, K)
    G = Phi.T @ Phi
    for t in range(20):
        theta = rng.dirichlet(0.3 * np.ones(K))
        n = rng.multinomial(int(rng.integers(3, 80)), Phi @ theta).astype(np.float64)
        w = n / n.sum()
        c = Phi.T @ w
        pi, _ = H.simplex_ls(G, c)
        ref = H.simplex_ls_bruteforce(G, c)
        assert np.abs(pi - ref).max() < 1e-10, (t, pi, ref)
        assert H.kkt_residual(G, c, pi) < 1e-10


def test_kkt_at_k100_and_both_kinds_of_optimum():
    rng = np.random.default_rng(7)
    V, K = 2000, 100
    Phi = _phi(rng, V, K, conc=0.01)
    G = Phi.T @ Phi
    sizes = []
    for t in range(10):
        theta = rng.dirichlet(0.1 * np.ones(K))
        n = rng.multinomial(150, Phi @ theta).astype(np.float64)
        c = Phi.T @ (n / n.sum())
        pi, _ = H.simplex_ls(G, c)
        assert H.kkt_residual(G, c, pi) < 1e-10
        sizes.append(int((pi > 0).sum()))
    assert min(sizes) >= 1 and max(sizes) > 1


def test_one_topic_document_is_fitted_exactly():
    rng = np.random.default_rng(9)
    V, K = 50, 6
    Phi = _phi(rng, V, K, conc=0.5)
    G = Phi.T @ Phi
    j = 4
    w = Phi[:, j]
    pi, _ = H.simplex_ls(G, Phi.T @ w)
    e = np.zeros(K)
    e[j] = 1.0
    assert np.abs(pi - e).max() < 1e-12

    class C:
        pass
    C.rowptr = np.array([0, V])
    C.col = np.arange(V)
    C.cnt = np.round(w * 1e6).astype(np.int64)   # integer counts close to w
    pis, lls = H.heldout_fit(C, Phi)
    n = C.cnt.astype(np.float64)
    ref_pi, _ = H.simplex_ls(G, Phi.T @ (n / n.sum()))
    assert np.abs(pis[0] - ref_pi).max() < 1e-12
    assert lls[0] == pytest.approx(float(np.sum(n * np.log(Phi @ ref_pi)) / n.sum()), rel=1e-14)
    assert abs(lls[0] - float(np.sum(w * np.log(Phi[:, j])))) < 1e-4


def test_fit_that_must_drop_an_index():
    """Columns (0.45, 0.45, 0.1), (1, 0, 0), (0, 1, 0) and target w =
    (0.6, 0.6, -0.1).  The nearest point of their hull is the midpoint of the
    last two columns: there the residual r = (-0.1, -0.1, 0.1) gives gradient
    Phi^T r = (-0.08, -0.1, -0.1), equal on the support and larger off it, so
    pi = (0, 1/2, 1/2).  The method starts at the first column (the best
    vertex), and the affine solution on all three columns puts a negative
    weight on it, so it has to take that index out again."""
    Phi = np.array([[0.45, 1.0, 0.0], [0.45, 0.0, 1.0], [0.1, 0.0, 0.0]])
    w = np.array([0.6, 0.6, -0.1])
    G, c = Phi.T @ Phi, Phi.T @ w
    assert int(np.argmin(0.5 * np.diag(G) - c)) == 0
    pi, it = H.simplex_ls(G, c)
    np.testing.assert_allclose(pi, [0.0, 0.5, 0.5], atol=1e-14)
    assert it >= 3
