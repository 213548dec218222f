"""Pins of the fast-ALS oracle (Appendix C, Algorithm 2) against what the
mathematics fixes, independent of the oracle's own code paths:

  * injective hashes (h_1(i) = i, h_2(j) = n j, h_3(k) = n^2 k, b >= n^3): the
    two-vector estimate of Proposition 1 equals the exact contraction, in all
    three read-off modes, for a non-symmetric tensor;
  * unbiasedness: averaged over every sign draw (and every hash draw on a tiny
    case) the estimate equals the exact contraction;
  * exact ALS recovers the factors of an exactly low-rank tensor;
  * with injective hashes sketched ALS is exact ALS;
  * the update with orthonormal other factors is the printed Algorithm 2 (no
    pseudo-inverse needed).
"""
import itertools

import numpy as np
import pytest

from oracle import als, sketch_dense


def _injective(n, rng):
    h = np.array([np.arange(n), n * np.arange(n), n * n * np.arange(n)], dtype=np.uint32)
    xi = rng.choice(np.array([-1, 1], dtype=np.int8), size=(3, n))
    return h, xi


@pytest.mark.parametrize("rd", [0, 1, 2])
def test_injective_hash_two_vector_contraction_is_exact(rd):
    rng = np.random.default_rng(rd)
    n = 5
    T = rng.standard_normal((n, n, n))           # not symmetric
    h, xi = _injective(n, rng)
    b = n ** 3
    s = sketch_dense(T, h, xi, b)
    X, Y = rng.standard_normal((3, n)), rng.standard_normal((3, n))
    got = als.contract_two(s, h, xi, X, Y, rd)
    # the exact contraction written out by loops
    ref = np.zeros((3, n))
    for r in range(3):
        for i, j, k in itertools.product(range(n), repeat=3):
            idx = (i, j, k)
            fixed = idx[rd]
            ref[r, fixed] += T[i, j, k] * X[r, idx[(rd + 1) % 3]] * Y[r, idx[(rd + 2) % 3]]
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(als.contract_two_dense(T, X, Y, rd), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("rd", [0, 1, 2])
def test_unbiased_over_all_sign_draws(rd):
    rng = np.random.default_rng(10 + rd)
    n, b = 3, 4                                   # collisions happen
    T = rng.standard_normal((n, n, n))
    h = rng.integers(0, b, size=(3, n)).astype(np.uint32)
    X, Y = rng.standard_normal((1, n)), rng.standard_normal((1, n))
    acc = np.zeros((1, n))
    cnt = 0
    for signs in itertools.product([-1, 1], repeat=3 * n):
        xi = np.array(signs, dtype=np.int8).reshape(3, n)
        acc += als.contract_two(sketch_dense(T, h, xi, b), h, xi, X, Y, rd)
        cnt += 1
    np.testing.assert_allclose(acc / cnt, als.contract_two_dense(T, X, Y, rd), rtol=0, atol=1e-12)


def test_unbiased_over_all_hash_and_sign_draws_tiny():
    rng = np.random.default_rng(3)
    n, b = 2, 2
    T = rng.standard_normal((n, n, n))
    X, Y = rng.standard_normal((1, n)), rng.standard_normal((1, n))
    acc = np.zeros((1, n))
    cnt = 0
    for hv in itertools.product(range(b), repeat=3 * n):
        h = np.array(hv, dtype=np.uint32).reshape(3, n)
        for signs in itertools.product([-1, 1], repeat=3 * n):
            xi = np.array(signs, dtype=np.int8).reshape(3, n)
            acc += als.contract_two(sketch_dense(T, h, xi, b), h, xi, X, Y, 0)
            cnt += 1
    np.testing.assert_allclose(acc / cnt, als.contract_two_dense(T, X, Y, 0), rtol=0, atol=1e-12)


def _planted(n, k, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    lam = np.linspace(2.0, 1.0, k)
    T = np.einsum("r,ir,jr,kr->ijk", lam, Q, Q, Q)
    return T, lam, Q.T, rng


def test_exact_als_recovers_low_rank_factors():
    n, k = 8, 3
    T, lam, V, rng = _planted(n, k, 1)
    F0 = np.stack([V + 0.1 * rng.standard_normal((k, n)) for _ in range(3)])
    r = als.als_dense(T, k, 30, F0)
    np.testing.assert_allclose(r.lam, lam, rtol=1e-10)
    for f in range(3):
        np.testing.assert_allclose(np.abs(np.sum(r.F[f] * V, axis=1)), 1.0, rtol=0, atol=1e-10)


def test_injective_sketched_als_equals_dense_als():
    n, k = 5, 2
    T, lam, V, rng = _planted(n, k, 2)
    T = T + 0.01 * rng.standard_normal((n, n, n))
    h, xi = _injective(n, rng)
    b = n ** 3
    S = sketch_dense(T, h, xi, b)[None]
    F0 = rng.standard_normal((3, k, n))
    rs = als.als_sketched(S, h[None], xi[None], k, 6, F0)
    rd = als.als_dense(T, k, 6, F0)
    np.testing.assert_allclose(rs.lam, rd.lam, rtol=1e-9)
    np.testing.assert_allclose(rs.F, rd.F, rtol=0, atol=1e-9)


def test_update_with_orthonormal_factors_is_the_printed_step():
    rng = np.random.default_rng(4)
    n, k = 7, 3
    X = np.linalg.qr(rng.standard_normal((n, k)))[0].T
    Y = np.linalg.qr(rng.standard_normal((n, k)))[0].T
    V = rng.standard_normal((k, n))
    lam, A = als.als_update(V, X, Y)
    np.testing.assert_allclose(lam, np.linalg.norm(V, axis=1), rtol=1e-12)
    np.testing.assert_allclose(A, V / np.linalg.norm(V, axis=1)[:, None], rtol=0, atol=1e-12)
