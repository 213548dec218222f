"""Pins of the colliding-hash symmetric sketch oracle (Section 3.3, Eq. (5);
Appendix B) against what the mathematics fixes:

  * for a symmetric tensor the sketch over all entries equals the sketch over
    i <= j <= k weighted by the number of index permutations (the section's
    cheap build);
  * averaged over every sign draw (all 4^n assignments of 4th roots of unity,
    any fixed hash) the entry recovery of Section 3.3, the T(u,u,u) estimate
    and the T(I,u,u) estimate are exactly unbiased -- and the T(I,u,u)
    read-off with the printed weights (1, 1/6, 1/6, 1) is not, which pins the
    1/3 on all four terms;
  * the FFT read-off equals the definition <s, s_{Z_i}>/3 by direct
    convolutions, and u . v(u) equals the T(u,u,u) estimate;
  * with all signs 1 and an injective hash into b > 3 max h the sketch holds
    each multiset's sum in its own bucket.
"""
import itertools

import numpy as np
import pytest

from oracle import symmetric as sy


def _sym_tensor(n, rng):
    A = rng.standard_normal((n, n, n))
    return sum(A.transpose(p) for p in itertools.permutations(range(3))) / 6


@pytest.mark.parametrize("seed", [0, 1])
def test_upper_triangle_build_equals_full_sum(seed):
    rng = np.random.default_rng(seed)
    n, b = 6, 11
    T = _sym_tensor(n, rng)
    h = rng.integers(0, b, n)
    q = rng.integers(0, 4, n)
    np.testing.assert_allclose(sy.sym_sketch_upper(T, h, q, b), sy.sym_sketch_dense(T, h, q, b),
                               rtol=0, atol=1e-12)


def test_unbiased_over_all_sign_draws_and_printed_weights_are_biased():
    rng = np.random.default_rng(2)
    n, b = 3, 5
    T = _sym_tensor(n, rng)
    h = rng.integers(0, b, n)
    u = rng.standard_normal(n)
    tuuu = np.einsum("ijk,i,j,k->", T, u, u, u)
    tiuu = np.einsum("ijk,j,k->i", T, u, u)
    acc_uuu, acc_iuu, acc_pr = 0.0, np.zeros(n, complex), np.zeros(n, complex)
    acc_rec = np.zeros((n, n, n), complex)
    sig_all = list(itertools.product(range(4), repeat=n))
    for qs in sig_all:
        q = np.array(qs)
        s = sy.sym_sketch_dense(T, h, q, b)
        acc_uuu += sy.sym_tuuu(s, h, q, u)
        acc_iuu += sy.sym_tiuu(s, h, q, u)
        acc_pr += sy.sym_tiuu(s, h, q, u, coef=(1.0, 1 / 6, 1 / 6, 1.0))
        sg = sy.sigma(q)
        for i, j, k in itertools.product(range(n), repeat=3):
            kappa = 1 if i == j == k else (3 if (i == j or j == k or i == k) else 6)
            acc_rec[i, j, k] += np.conj(sg[i] * sg[j] * sg[k]) * s[(h[i] + h[j] + h[k]) % b] / kappa
    N = len(sig_all)
    assert abs(acc_uuu / N - tuuu) < 1e-12
    np.testing.assert_allclose(acc_iuu / N, tiuu, rtol=0, atol=1e-12)
    np.testing.assert_allclose(acc_rec / N, T, rtol=0, atol=1e-12)
    assert np.max(np.abs(acc_pr / N - tiuu)) > 1e-3


def test_fft_read_off_equals_definition_and_uuu_identity():
    rng = np.random.default_rng(3)
    n, b = 5, 16
    T = _sym_tensor(n, rng)
    h = rng.integers(0, b, n)
    q = rng.integers(0, 4, n)
    u = rng.standard_normal(n)
    s = sy.sym_sketch_dense(T, h, q, b)
    v = sy.sym_tiuu(s, h, q, u)
    np.testing.assert_allclose(v, sy.sym_tiuu_direct(s, h, q, u), rtol=0, atol=1e-12)
    assert abs(u @ v - sy.sym_tuuu(s, h, q, u)) < 1e-12


def test_injective_hash_separates_multisets():
    rng = np.random.default_rng(4)
    n = 4
    T = _sym_tensor(n, rng)
    h = np.array([0, 1, 4, 13])          # all sums h_i + h_j + h_k of multisets distinct
    b = 64
    s = sy.sym_sketch_dense(T, h, np.zeros(n, int), b)
    for i, j, k in itertools.combinations_with_replacement(range(n), 3):
        mult = 1 if i == j == k else (3 if (i == j or j == k) else 6)
        assert abs(s[h[i] + h[j] + h[k]] - mult * T[i, j, k]) < 1e-12
