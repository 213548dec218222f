"""Parity of fast ALS (Appendix C, Algorithm 2) with the oracle, through the
C ABI: the two-vector contraction in all three read-off modes, single ALS
sweeps and whole runs (FP64 and FP32 power steps), a singular Gram matrix
(pseudo-inverse), recovery of planted factors, argument errors.

Bars: FP64 contractions 1e-12 normwise relative, FP32 ones 1e-5.  An ALS
update solves with the k x k Gram matrix G = (X X^T) o (Y Y^T), which
multiplies the relative error of its inputs by up to cond(G); whole runs are
held to 1e-12 (FP64) and 1e-5 (FP32) times the largest cond(G) of the
oracle's run (printed with the observed error).
Inputs: seeded planted symmetric tensors with noise, random start factors.
"""
import numpy as np
import pytest

import oracle
from oracle import als as oals
from paper_1506_04448_amd.workloads import planted_tensor

torch = pytest.importorskip("torch")
import paper_1506_04448_amd as tsk  # noqa: E402
from parity_rules import rel  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gram_conditioning(S_time, h, xi, k, T, F0):
    """Largest cond(G) over the updates of the oracle's ALS run (the same
    iteration as oracle.als.als_sketched, stepped update by update here to
    read each G)."""
    F = np.array(F0, dtype=np.float64, copy=True)
    B = S_time.shape[0]
    kmax = 1.0
    for _ in range(T):
        for rd in range(3):
            X, Y = F[(rd + 1) % 3], F[(rd + 2) % 3]
            G = (X @ X.T) * (Y @ Y.T)
            ev = np.abs(np.linalg.eigvalsh(G))
            keep = ev > 1e-12 * ev.max()
            kmax = max(kmax, float(ev[keep].max() / ev[keep].min()))
            V = np.stack([oals.contract_two(S_time[m], h[m], xi[m], X, Y, rd) for m in range(B)], axis=1)
            _, F[rd] = oals.als_update(oracle.median(V, axis=1), X, Y)
    return kmax


def check_als(lam, F, ref, base, kappa, label):
    el, ef = rel(lam, ref.lam), rel(F, ref.F)
    bar = base * kappa
    print(f"{label}: lambda rel err {el:.2e}, factors rel err {ef:.2e}, max cond(G) {kappa:.1f}, "
          f"bar {bar:.1e}", flush=True)
    assert el < bar and ef < bar, (el, ef, bar)


@pytest.fixture(scope="module")
def ctx():
    c = tsk.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _setup(ctx, n, k, b, B, seed, dt=np.float64):
    P = planted_tensor(n, k, noise=0.02, seed=seed, dtype=dt)
    h, xi = tsk.hash_generate(seed + 100, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    S_time = np.stack([oracle.sketch_dense(P.T.astype(np.float64), h[m], xi[m], b) for m in range(B)])
    return P, tab, h, xi, S64, S32, S_time


@pytest.mark.parametrize("n,b,B,L,dtype,tol", [
    (40, 1024, 3, 5, torch.float64, 1e-12),
    (37, 256, 4, 3, torch.float64, 1e-12),
    (200, 16384, 4, 6, torch.float32, 1e-5),
    (90, 32768, 2, 3, torch.float32, 1e-5),
    (150, 8192, 3, 4, torch.float64, 1e-12),
    (120, 65536, 2, 3, torch.float32, 1e-5),
])
def test_contract_two_matches_oracle(ctx, n, b, B, L, dtype, tol):
    print(f"contract_two n={n} b={b} B={B} {dtype}", flush=True)
    P, tab, h, xi, S64, S32, S_time = _setup(ctx, n, 3, b, B, 7)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((L, n))
    Y = rng.standard_normal((L, n))
    if dtype == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
        Y = Y.astype(np.float32).astype(np.float64)
    for rd in range(3):
        V = tsk.contract_two(ctx, tab, torch.from_numpy(X).to(DEV, dtype), torch.from_numpy(Y).to(DEV, dtype),
                             rd=rd, S64=S64, S32=S32).cpu().numpy()
        for m in range(B):
            ref = oals.contract_two(S_time[m], h[m], xi[m], X, Y, rd)
            assert rel(V[:, m], ref) < tol, (rd, m, rel(V[:, m], ref))


@pytest.mark.parametrize("B", [3, 4, 20])
def test_als_sweeps_fp64_match_oracle(ctx, B):
    print(f"als fp64 B={B}", flush=True)
    n, k, b = 30, 3, 1024
    P, tab, h, xi, S64, S32, S_time = _setup(ctx, n, k, b, B, 3)
    rng = np.random.default_rng(B)
    F0 = rng.standard_normal((3, k, n))
    for T in (1, 6):
        lam, F = tsk.als(ctx, tab, torch.from_numpy(F0).to(DEV), T, dtype=tsk.F64, S64=S64)
        ref = oals.als_sketched(S_time, h, xi, k, T, F0)
        check_als(lam.cpu().numpy(), F.cpu().numpy(), ref, 1e-12,
                  gram_conditioning(S_time, h, xi, k, T, F0), f"als fp64 B={B} T={T}")


def test_als_fp32_matches_oracle(ctx):
    n, k, b, B = 100, 4, 16384, 5
    P, tab, h, xi, S64, S32, S_time = _setup(ctx, n, k, b, B, 4, dt=np.float32)
    rng = np.random.default_rng(9)
    F0 = rng.standard_normal((3, k, n))
    lam, F = tsk.als(ctx, tab, torch.from_numpy(F0).to(DEV), 3, dtype=tsk.F32, S32=S32)
    ref = oals.als_sketched(S_time, h, xi, k, 3, F0)
    check_als(lam.cpu().numpy(), F.cpu().numpy(), ref, 1e-5,
              gram_conditioning(S_time, h, xi, k, 3, F0), "als fp32 b=16384")


def test_als_singular_gram_uses_pseudo_inverse(ctx):
    """Two equal start columns in every factor: G is singular after the
    first update of each sweep, and the pseudo-inverse decides the result."""
    n, k, b, B = 25, 3, 512, 3
    P, tab, h, xi, S64, S32, S_time = _setup(ctx, n, k, b, B, 5)
    rng = np.random.default_rng(2)
    F0 = rng.standard_normal((3, k, n))
    F0[:, 2] = F0[:, 1]
    lam, F = tsk.als(ctx, tab, torch.from_numpy(F0).to(DEV), 1, dtype=tsk.F64, S64=S64)
    ref = oals.als_sketched(S_time, h, xi, k, 1, F0)
    check_als(lam.cpu().numpy(), F.cpu().numpy(), ref, 1e-12,
              gram_conditioning(S_time, h, xi, k, 1, F0), "als singular Gram")


def test_als_recovers_planted_factors(ctx):
    n, k, b, B = 60, 4, 8192, 8
    P, tab, h, xi, S64, S32, S_time = _setup(ctx, n, k, b, B, 6, dt=np.float32)
    rng = np.random.default_rng(6)
    F0 = np.stack([P.V + 0.3 * rng.standard_normal((k, n)) for _ in range(3)])
    lam, F = tsk.als(ctx, tab, torch.from_numpy(F0).to(DEV), 15, dtype=tsk.F32, S32=S32)
    lam, F = lam.cpu().numpy(), F.cpu().numpy()
    for f in range(3):
        assert oracle.wrong_vectors(P.V, F[f]) == 0
    np.testing.assert_allclose(np.sort(lam), np.sort(P.lam), rtol=0.05)


def test_als_fp32_split_transforms_match_oracle(ctx):
    """b = 65536: the power steps run through the split transforms."""
    n, k, b, B = 50, 3, 65536, 2
    P, tab, h, xi, S64, S32, S_time = _setup(ctx, n, k, b, B, 8, dt=np.float32)
    rng = np.random.default_rng(8)
    F0 = rng.standard_normal((3, k, n))
    lam, F = tsk.als(ctx, tab, torch.from_numpy(F0).to(DEV), 2, dtype=tsk.F32, S32=S32)
    ref = oals.als_sketched(S_time, h, xi, k, 2, F0)
    check_als(lam.cpu().numpy(), F.cpu().numpy(), ref, 1e-5,
              gram_conditioning(S_time, h, xi, k, 2, F0), "als fp32 b=65536")


def test_als_argument_errors(ctx):
    h, xi = tsk.hash_generate(1, 10, 65536, 2)
    tab = tsk.Tables(ctx, h, xi, 65536)
    S64, S32 = tsk.new_sketch(tab, DEV)
    F0 = torch.zeros((3, 2, 10), dtype=torch.float64, device=DEV)
    with pytest.raises(tsk.TskError, match="EUNSUPPORTED"):
        tsk.als(ctx, tab, F0, 1, dtype=tsk.F64, S64=S64)
    X = torch.zeros((2, 10), dtype=torch.float64, device=DEV)
    with pytest.raises(tsk.TskError, match="EUNSUPPORTED"):
        tsk.contract_two(ctx, tab, X, X, S64=S64)
    tab.close()
    h, xi = tsk.hash_generate(1, 10, 256, 2)
    tab = tsk.Tables(ctx, h, xi, 256)
    S64, S32 = tsk.new_sketch(tab, DEV)
    with pytest.raises(tsk.TskError, match="k=65"):
        tsk.als(ctx, tab, torch.zeros((3, 65, 10), dtype=torch.float64, device=DEV), 1, dtype=tsk.F64, S64=S64)
    with pytest.raises(tsk.TskError, match="T=0"):
        tsk.als(ctx, tab, F0, 0, dtype=tsk.F64, S64=S64)
    X = torch.zeros((2, 10), dtype=torch.float64, device=DEV)
    with pytest.raises(tsk.TskError, match="rd=3"):
        tsk.contract_two(ctx, tab, X, X, rd=3, S64=S64)
