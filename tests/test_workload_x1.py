"""The synthetic full-rank tensors of the paper's accuracy table (Section 5.1,
Table 5), built by `workloads.full_rank_tensor`: structure checks at small n,
and the noise-level reading pinned by the printed exact residuals.

Reading: the paper writes the noise as N(0, sigma/n^1.5) and calls sigma the
noise-to-signal level.  For the normalised full-rank signal the squared
residual of the exact top-10 recovery is sum_{i>10} lam_i^2 + ||E||_F^2
(E is almost orthogonal to the ten components), and the printed exact
residuals, 0.07 at sigma = 0.01 and 0.16 at sigma = 0.1, match
E||E||_F^2 = sigma (variance sigma/n^3 per entry) and not ||E||_F = sigma.
"""
import os

import numpy as np
import pytest

from paper_1506_04448_amd.workloads import full_rank_tensor

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table5_exact.txt")


def _exact_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            if len(f) == 3:
                rows.append((float(f[0]), float(f[1]), int(f[2])))
    return rows


def test_structure_small():
    n = 11
    X = full_rank_tensor(n, 0.05, seed=4, chunk=4)
    T = X.T.double().numpy()
    for p in [(0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0), (2, 0, 1)]:
        assert np.array_equal(T, T.transpose(p))
    np.testing.assert_allclose(X.V @ X.V.T, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(X.lam[0] / X.lam[4], 5.0, rtol=1e-12)
    assert abs(np.sum(X.lam ** 2) - 1.0) < 1e-12
    S = np.einsum("r,ri,rj,rk->ijk", X.lam, X.V, X.V, X.V)
    assert abs(np.linalg.norm(S) - 1.0) < 1e-12
    # without noise the tensor is the FP32 rounding of the signal
    X0 = full_rank_tensor(n, 0.0, seed=4, chunk=4)
    np.testing.assert_allclose(X0.T.double().numpy(), S, atol=1e-7)
    # the noise copies one value to all permutations of each index triple
    E = T - X0.T.double().numpy()
    assert np.isclose(E[1, 2, 3], E[3, 1, 2]) and np.isclose(E[0, 0, 5], E[5, 0, 0])


def test_noise_level_is_expected_squared_norm():
    n, sigma = 14, 0.1
    # independent entries i<=j<=k with multiplicities: E||E||^2 = sigma exactly
    vals = []
    for seed in range(12):
        X = full_rank_tensor(n, sigma, seed=seed, chunk=7)
        X0 = full_rank_tensor(n, 0.0, seed=seed, chunk=7)
        vals.append(float(((X.T.double() - X0.T.double()) ** 2).sum()))
    m = float(np.mean(vals))
    assert abs(m - sigma) < 0.1 * sigma, m


@pytest.mark.parametrize("sigma,printed,wrong", _exact_rows())
def test_noise_reading_matches_printed_exact_residuals(sigma, printed, wrong):
    n = 1000
    lam = 1.0 / np.arange(1, n + 1)
    lam2 = lam ** 2 / np.sum(lam ** 2)
    tail = float(np.sum(lam2[10:]))
    # the reading: E||E||^2 = sigma -> residual tail + sigma, within the 2 printed digits
    assert abs(tail + sigma - printed) < 0.006
    # the other reading (standard deviation sigma / n^1.5, ||E||^2 ~ sigma^2) misses sigma = 0.1
    if sigma >= 0.1:
        assert abs(tail + sigma ** 2 - printed) > 0.05
    assert wrong == 0
