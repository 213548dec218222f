"""Held-out likelihood of a topic model (Section 5.2) -- test infrastructure only.

A topic matrix Phi (V x K, columns on the simplex) is scored on held-out
documents.  For a document with word counts n (length m) and empirical word
distribution w = n / m, the mixing vector is the simplex-constrained least
squares fit

    pi_hat = argmin { ||w - Phi pi||_2 : pi >= 0, sum_k pi_k = 1 },

and the document's score is the average log-probability of its words,

    L_d = (1/m) sum_i n_i ln( sum_k pi_hat_k Phi[i, k] ).

With G = Phi^T Phi and c = Phi^T w the fit minimises (1/2) pi^T G pi - c^T pi
over the simplex, a convex quadratic programme.  It is solved exactly by the
primal active-set method for convex quadratic programmes (Nocedal and Wright,
Numerical Optimization, Sec. 16.5): on the current free set F the
equality-constrained problem min (1/2) x^T G_FF x - c_F^T x, 1^T x = 1 has the
KKT system [G_FF 1; 1^T 0] [x; nu] = [c_F; 1]; a solution with x >= 0 is
accepted and the multipliers mu_k = (G pi - c)_k + nu of the indices held at
zero decide whether one of them enters F (the most negative, lowest index on
ties); otherwise the step towards x stops at the first index reaching zero,
which leaves F.

Pinned by tests/test_oracle_heldout_pins.py: the active-set result equals the
best of the equality-constrained solutions over every support (brute force,
K <= 7), satisfies the KKT conditions at K = 100, and the likelihood reduces
to the closed form for one-topic documents.
"""
from __future__ import annotations

import itertools

import numpy as np


def _eq_qp(G: np.ndarray, c: np.ndarray):
    """x, nu with G x + nu 1 = c and 1^T x = 1."""
    f = len(c)
    A = np.zeros((f + 1, f + 1))
    A[:f, :f] = G
    A[:f, f] = 1.0
    A[f, :f] = 1.0
    rhs = np.concatenate([c, [1.0]])
    sol = np.linalg.solve(A, rhs)
    return sol[:f], sol[f]


def simplex_ls(G: np.ndarray, c: np.ndarray, max_iter: int = 1000):
    """argmin of (1/2) pi^T G pi - c^T pi over the simplex by the primal
    active-set method (G symmetric positive definite).  Returns (pi, iterations)."""
    K = len(c)
    tol = 1e-12 * float(np.max(np.diag(G)))
    j = int(np.argmin(0.5 * np.diag(G) - c))       # best vertex
    free = [j]
    pi = np.zeros(K)
    pi[j] = 1.0
    for it in range(1, max_iter + 1):
        F = sorted(free)
        x, nu = _eq_qp(G[np.ix_(F, F)], c[F])
        if np.all(x >= 0.0):
            pi[:] = 0.0
            pi[F] = x
            mu = G @ pi - c + nu
            mu[F] = np.inf
            k = int(np.argmin(mu))
            if mu[k] >= -tol:
                return pi, it
            free.append(k)
        else:
            cur = pi[F]
            ratios = np.full(len(F), np.inf)
            neg = x < 0.0
            ratios[neg] = cur[neg] / (cur[neg] - x[neg])
            a = int(np.argmin(ratios))
            pi[F] = cur + ratios[a] * (x - cur)
            pi[F[a]] = 0.0
            free.remove(F[a])
    raise RuntimeError("simplex_ls: no convergence")


def simplex_ls_bruteforce(G: np.ndarray, c: np.ndarray) -> np.ndarray:
    """The same argmin by trying every support: the equality-constrained
    solution on each support, kept when it is non-negative, the best kept."""
    K = len(c)
    best, best_val = None, np.inf
    for r in range(1, K + 1):
        for S in itertools.combinations(range(K), r):
            S = list(S)
            x, _ = _eq_qp(G[np.ix_(S, S)], c[S])
            if np.all(x >= -1e-14):
                pi = np.zeros(K)
                pi[S] = np.maximum(x, 0.0)
                val = 0.5 * pi @ G @ pi - c @ pi
                if val < best_val:
                    best, best_val = pi, val
    return best


def kkt_residual(G: np.ndarray, c: np.ndarray, pi: np.ndarray) -> float:
    """Largest violation of the optimality conditions of the simplex
    programme at pi, relative to max diag G: feasibility (pi >= 0, sum 1), and
    with g = G pi - c, g_k equal to its minimum over the support and not below
    it elsewhere."""
    g = G @ pi - c
    supp = pi > 0.0
    gmin = g[supp].min()
    scale = float(np.max(np.diag(G)))
    viol = max(-pi.min(), abs(pi.sum() - 1.0))
    viol = max(viol, float(np.max(np.abs(g[supp] - gmin))) / scale)
    viol = max(viol, float(max(0.0, -(g[~supp] - gmin).min() if (~supp).any() else 0.0)) / scale)
    return viol


def heldout_fit(corpus, Phi: np.ndarray, docs=None):
    """pi_hat [D][K] and L_d [D] for the documents of `corpus` (CSR rowptr,
    col, cnt) under the topic matrix Phi [V][K]; `docs` selects documents."""
    G = Phi.T @ Phi
    ids = range(len(corpus.rowptr) - 1) if docs is None else docs
    pis, lls = [], []
    for d in ids:
        lo, hi = corpus.rowptr[d], corpus.rowptr[d + 1]
        words = corpus.col[lo:hi]
        n = corpus.cnt[lo:hi].astype(np.float64)
        m = n.sum()
        c = Phi[words].T @ (n / m)
        pi, _ = simplex_ls(G, c)
        p = Phi[words] @ pi
        pis.append(pi)
        lls.append(float(np.sum(n * np.log(p)) / m))
    return np.array(pis), np.array(lls)
