"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: tables bit-exact (host tests); FP64 steps within 1e-12 normwise
relative; FP32 steps within 1e-5 normwise relative.
Inputs are seeded and synthetic (planted symmetric tensors, see
paper_1506_04448_amd/workloads.py); the oracle builds its own sketches from the
same tensor with its own tables unless a test isolates a single step.
"""
import numpy as np
import pytest

import oracle
from paper_1506_04448_amd.workloads import planted_tensor

torch = pytest.importorskip("torch")
import paper_1506_04448_amd as tsk  # noqa: E402
from parity_rules import near_tie, rel  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"




@pytest.fixture(scope="module")
def ctx():
    c = tsk.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _tables(ctx, seed, n, b, B):
    h, xi = tsk.hash_generate(seed, n, b, B)
    return tsk.Tables(ctx, h, xi, b), h, xi


def _time_sketch(ctx, tab, S64):
    return tsk.sketch_export(ctx, S64, tab.b).cpu().numpy()


def _oracle_sketches(T, h, xi, b):
    return np.stack([oracle.sketch_dense(T, h[m], xi[m], b) for m in range(h.shape[0])])


def _gpu_spectra_from(ctx, tab, S_time):
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_from_time(ctx, torch.from_numpy(S_time).to(DEV), S64, S32)
    return S64, S32


# ----------------------------------------------------------------------------- build

@pytest.mark.parametrize("n,b,B,dtype", [(50, 1024, 4, np.float64), (37, 256, 3, np.float64),
                                         (37, 256, 3, np.float32), (1, 64, 1, np.float64),
                                         (65, 8192, 5, np.float32), (300, 4096, 8, np.float32),
                                         (120, 16384, 3, np.float64)])
def test_dense_build_matches_eq1(ctx, n, b, B, dtype):
    print(f"build n={n} b={b} B={B} {np.dtype(dtype).name}", flush=True)
    P = planted_tensor(n, min(3, n), noise=0.05, seed=n, dtype=dtype)
    tab, h, xi = _tables(ctx, 11, n, b, B)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    got = _time_sketch(ctx, tab, S64)
    ref = _oracle_sketches(P.T.astype(np.float64), h, xi, b)
    tol = 1e-12 if dtype == np.float64 else 1e-5
    for m in range(B):
        assert rel(got[m], ref[m]) < tol, (m, rel(got[m], ref[m]))
    # working copy is the master rounded to FP32
    np.testing.assert_array_equal(S32.cpu().numpy(), S64.cpu().numpy().astype(np.float32))


def test_dense_build_full_size_c2(ctx):
    n, b, B = 200, 16384, 10
    P = planted_tensor(n, 10, noise=0.05, seed=1, dtype=np.float32)
    tab, h, xi = _tables(ctx, 1, n, b, B)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    got = _time_sketch(ctx, tab, S64)
    T64 = P.T.astype(np.float64)
    for m in (0, 9):
        ref = oracle.sketch_dense(T64, h[m], xi[m], b)
        assert rel(got[m], ref) < 1e-5, (m, rel(got[m], ref))
    # linearity: accumulate doubles the spectrum
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32, accumulate=True)
    got2 = _time_sketch(ctx, tab, S64)
    assert rel(got2, 2 * got) < 1e-6


@pytest.mark.parametrize("n,b,B,dtype", [(40, 1024, 6, np.float32), (200, 16384, 2, np.float32),
                                         (33, 32768, 2, np.float64), (3, 64, 2, np.float32)])
def test_dense_build_of_integer_tensor_is_exact(ctx, n, b, B, dtype):
    """Small integer entries make every bin sum exact on both sides, so the
    fixed-point build (signs, bins, scale) must equal Eq. (1) up to the FP64
    transform round trip of the export; the tensor is not symmetric, so each
    mode's table is checked against its own index."""
    print(f"exact build n={n} b={b} B={B} {np.dtype(dtype).name}", flush=True)
    rng = np.random.default_rng(n + b)
    T = rng.integers(-7, 8, size=(n, n, n)).astype(dtype)
    tab, h, xi = _tables(ctx, 23, n, b, B)
    S64, S32 = tsk.new_sketch(tab, DEV)
    Td = torch.from_numpy(T).to(DEV)
    tsk.sketch_build_dense(ctx, tab, Td, S64, S32)
    got = _time_sketch(ctx, tab, S64)
    ref = _oracle_sketches(T.astype(np.float64), h, xi, b)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9)
    # rebuilding gives the same bits (integer sums do not depend on order)
    S64b, S32b = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, Td, S64b, S32b)
    np.testing.assert_array_equal(S64b.cpu().numpy(), S64.cpu().numpy())


def test_spectrum_roundtrip_matches_numpy_fft(ctx):
    rng = np.random.default_rng(0)
    for b, B in [(64, 1), (1024, 3), (16384, 2)]:
        s = rng.standard_normal((B, b))
        S64 = torch.zeros((B, b // 2 + 1, 2), dtype=torch.float64, device=DEV)
        S32 = torch.zeros((B, b // 2 + 1, 2), dtype=torch.float32, device=DEV)
        tsk.sketch_from_time(ctx, torch.from_numpy(s).to(DEV), S64, S32)
        spec = S64.cpu().numpy()
        ref = np.fft.rfft(s, axis=-1)
        assert rel(spec[..., 0] + 1j * spec[..., 1], ref) < 1e-14
        back = tsk.sketch_export(ctx, S64, b).cpu().numpy()
        assert rel(back, s) < 1e-14


# ----------------------------------------------------------------------------- steps

@pytest.mark.parametrize("n,b,B,L,dtype,tol", [
    (50, 1024, 4, 6, torch.float64, 1e-12),
    (50, 1024, 5, 3, torch.float64, 1e-12),
    (200, 16384, 10, 8, torch.float32, 1e-5),
    (37, 2048, 3, 5, torch.float32, 1e-5),
    (1, 64, 1, 2, torch.float64, 1e-12),
    (300, 8192, 64, 2, torch.float64, 1e-12),
])
def test_power_update_matches_prop1(ctx, n, b, B, L, dtype, tol):
    print(f"power n={n} b={b} B={B} L={L} {dtype}", flush=True)
    P = planted_tensor(n, min(4, n), noise=0.05, seed=2)
    tab, h, xi = _tables(ctx, 5, n, b, B)
    S_time = _oracle_sketches(P.T, h, xi, b)
    S64, S32 = _gpu_spectra_from(ctx, tab, S_time)
    rng = np.random.default_rng(3)
    U = rng.standard_normal((L, n))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    if dtype == torch.float32:
        U = U.astype(np.float32).astype(np.float64)   # the GPU sees exactly these values
    Ud = torch.from_numpy(U).to(device=DEV, dtype=dtype)
    V = torch.empty((L, B, n), dtype=dtype, device=DEV)
    flags = torch.zeros((L,), dtype=torch.int32, device=DEV)
    Uo = tsk.power_update(ctx, tab, Ud, S64=S64, S32=S32, V=V, flags=flags)
    Vr, Ur, fr = oracle.power_update(S_time, h, xi, U)
    Vg = V.cpu().numpy()
    for tau in range(L):
        for m in range(B):
            assert rel(Vg[tau, m], Vr[tau, m]) < tol, (tau, m, rel(Vg[tau, m], Vr[tau, m]))
    assert rel(Uo.cpu().numpy(), Ur) < tol
    assert flags.cpu().numpy().tolist() == fr.tolist()


@pytest.mark.parametrize("n,b,B,L,dtype,tol", [
    (200, 16384, 10, 50, torch.float32, 1e-5),
    (50, 16384, 3, 4, torch.float64, 1e-12),
    (2000, 4096, 8, 3, torch.float32, 1e-5),
    (512, 16384, 2, 3, torch.float32, 1e-5),
    (513, 16384, 2, 3, torch.float32, 1e-5),
])
def test_contract_tiuu_per_sketch(ctx, n, b, B, L, dtype, tol):
    """Proposition 1 per sketch, no median (the launch the benchmark times); n = 512 and 513
    sit on both sides of the bound below which the inverse leaves out its last two passes."""
    print(f"tiuu n={n} b={b} B={B} L={L} {dtype}", flush=True)
    rng = np.random.default_rng(12)
    tab, h, xi = _tables(ctx, 13, n, b, B)
    S_time = rng.standard_normal((B, b))
    S64, S32 = _gpu_spectra_from(ctx, tab, S_time)
    U = rng.standard_normal((L, n))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    if dtype == torch.float32:
        U = U.astype(np.float32).astype(np.float64)
    V = tsk.contract_tiuu(ctx, tab, torch.from_numpy(U).to(device=DEV, dtype=dtype), S64=S64, S32=S32)
    Vg = V.cpu().numpy()
    for m in range(B):
        ref = oracle.power_update_sketch(S_time[m], h[m], xi[m], U)
        for tau in range(L):
            assert rel(Vg[tau, m], ref[tau]) < tol, (tau, m, rel(Vg[tau, m], ref[tau]))


@pytest.mark.parametrize("n,b,B,L,dtype,tol", [
    (50, 1024, 4, 6, torch.float64, 1e-12),
    (200, 16384, 10, 8, torch.float32, 1e-5),
    (20, 512, 7, 3, torch.float32, 1e-5),
])
def test_contract_uuu_matches_eq3(ctx, n, b, B, L, dtype, tol):
    P = planted_tensor(n, 3, noise=0.05, seed=4)
    tab, h, xi = _tables(ctx, 6, n, b, B)
    S_time = _oracle_sketches(P.T, h, xi, b)
    S64, S32 = _gpu_spectra_from(ctx, tab, S_time)
    rng = np.random.default_rng(5)
    U = rng.standard_normal((L, n))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    if dtype == torch.float32:
        U = U.astype(np.float32).astype(np.float64)
    lam_med, lam_per = tsk.contract_uuu(ctx, tab, torch.from_numpy(U).to(device=DEV, dtype=dtype),
                                        S64=S64, S32=S32)
    per_r, med_r = oracle.contract_uuu(S_time, h, xi, U)
    scale = np.abs(per_r).max()
    assert np.abs(lam_per.cpu().numpy() - per_r).max() / scale < tol
    assert np.abs(lam_med.cpu().numpy() - med_r).max() / scale < tol


def test_deflate_matches_linearity(ctx):
    n, b, B = 40, 2048, 3
    P = planted_tensor(n, 3, noise=0.05, seed=7)
    tab, h, xi = _tables(ctx, 8, n, b, B)
    S_time = _oracle_sketches(P.T, h, xi, b)
    S64, S32 = _gpu_spectra_from(ctx, tab, S_time)
    lam = np.array([1.3, -0.4])
    U = P.V[:2].copy()
    tsk.sketch_deflate(ctx, tab, torch.from_numpy(lam).to(DEV), torch.from_numpy(U).to(DEV), S64, S32)
    got = _time_sketch(ctx, tab, S64)
    for m in range(B):
        ref = S_time[m] - sum(lam[r] * oracle.sketch_rank1_fft(U[r], U[r], U[r], h[m], xi[m], b)
                              for r in range(2))
        assert rel(got[m], ref) < 1e-12
    np.testing.assert_array_equal(S32.cpu().numpy(), S64.cpu().numpy().astype(np.float32))


@pytest.mark.parametrize("n,k,b,B", [(40, 5, 2048, 3), (150, 20, 16384, 2), (7, 1, 64, 1)])
def test_factor_build_matches_eq2(ctx, n, k, b, B):
    rng = np.random.default_rng(n)
    lam = rng.uniform(1, 10, k)
    A = rng.standard_normal((k, n))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    tab, h, xi = _tables(ctx, 9, n, b, B)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_factors(ctx, tab, torch.from_numpy(lam).to(DEV), torch.from_numpy(A).to(DEV),
                             S64, S32)
    got = _time_sketch(ctx, tab, S64)
    for m in range(B):
        ref = oracle.sketch_factors(lam, A, h[m], xi[m], b)
        assert rel(got[m], ref) < 1e-12, (m, rel(got[m], ref))


def _factor_sketches(ctx, seed, n, k, b, B):
    """Factor build (Eq. (2)) of a random rank-k tensor on the GPU and in the oracle."""
    rng = np.random.default_rng(seed)
    lam = rng.uniform(1, 10, k)
    A = rng.standard_normal((k, n))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    tab, h, xi = _tables(ctx, seed, n, b, B)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_factors(ctx, tab, torch.from_numpy(lam).to(DEV), torch.from_numpy(A).to(DEV),
                             S64, S32)
    S_time = np.stack([oracle.sketch_factors(lam, A, h[m], xi[m], b) for m in range(B)])
    return tab, h, xi, S64, S32, S_time


# The largest n a power step takes: n = 65535 through the split transforms
# (b = 65536); below that the work-group's LDS (half spectrum and u) bounds n,
# exactly at 19348 (FP64, b = 1024) and 23252 (FP32, b = 16384).
@pytest.mark.parametrize("b,dtype,tol,n_max", [(1024, torch.float64, 1e-12, 19348),
                                                (16384, torch.float32, 1e-5, 23252),
                                                (65536, torch.float32, 1e-5, 65535)])
def test_largest_n_factor_build_and_power_step(ctx, b, dtype, tol, n_max):
    """n = 65535 (the largest dimension the tables take) through the factor build, then one
    power step (Prop. 1 per sketch, the median and normalisation) at the largest n it
    supports, far above what one work-group stages for a fused median; one more
    coordinate is refused."""
    B, L = 3, 2
    print(f"largest n b={b} {dtype} n_max={n_max}", flush=True)
    tab, h, xi, S64, S32, S_time = _factor_sketches(ctx, b + 7, 65535, 3, b, B)
    assert rel(_time_sketch(ctx, tab, S64), S_time) < 1e-12
    if n_max < 65535:
        tab, h, xi, S64, S32, S_time = _factor_sketches(ctx, b + 8, n_max, 3, b, B)
        t2, _, _ = _tables(ctx, 3, n_max + 1, b, B)
        S64b, S32b = tsk.new_sketch(t2, DEV)
        with pytest.raises(tsk.TskError, match="LDS"):
            tsk.power_update(ctx, t2, torch.zeros((L, n_max + 1), dtype=dtype, device=DEV),
                             S64=S64b, S32=S32b)
    rng = np.random.default_rng(b)
    U = rng.standard_normal((L, n_max))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    if dtype == torch.float32:
        U = U.astype(np.float32).astype(np.float64)
    V = torch.empty((L, B, n_max), dtype=dtype, device=DEV)
    Uo = tsk.power_update(ctx, tab, torch.from_numpy(U).to(device=DEV, dtype=dtype),
                          S64=S64, S32=S32, V=V)
    Vr, Ur, _ = oracle.power_update(S_time, h, xi, U)
    Vg = V.cpu().numpy()
    for tau in range(L):
        for m in range(B):
            assert rel(Vg[tau, m], Vr[tau, m]) < tol, (tau, m, rel(Vg[tau, m], Vr[tau, m]))
    assert rel(Uo.cpu().numpy(), Ur) < tol


# ----------------------------------------------------------------------------- decompose

def test_decompose_fp64_small_config(ctx):
    """n=50 FP64, b=1024, B=4, L=10, T=20, k=5, seed 0: the whole of Algorithm 1."""
    n, k, b, B, L, T = 50, 5, 1024, 4, 10, 20
    P = planted_tensor(n, 5, noise=0.01, seed=0)
    tab, h, xi = _tables(ctx, 0, n, b, B)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    u0 = np.stack([oracle.start_vectors_spec(0, c, L, n) for c in range(k)])
    lam, U, tau, flags = tsk.decompose(ctx, tab, S64, S32, k, L, T, dtype=tsk.F64,
                                       u0=torch.from_numpy(u0).to(DEV))
    ref = oracle.rtpm_sketched(_oracle_sketches(P.T, h, xi, b), h, xi, k, L, T, u0)
    assert rel(lam.cpu().numpy(), ref.lam) < 1e-12
    assert rel(U.cpu().numpy(), ref.U) < 1e-12
    np.testing.assert_array_equal(flags.cpu().numpy(), ref.flags)
    assert rel(_time_sketch(ctx, tab, S64), ref.S) < 1e-12
    # null u0: the library draws the start vectors from the same spec
    S64b, S32b = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64b, S32b)
    lam2, U2, _, _ = tsk.decompose(ctx, tab, S64b, S32b, k, L, T, dtype=tsk.F64, seed=0)
    assert rel(lam2.cpu().numpy(), ref.lam) < 1e-12
    assert rel(U2.cpu().numpy(), ref.U) < 1e-12


def check_fp32_decomposition(ref, lam, U, S64_time, S_in, h, xi, b, label):
    """Every component of an FP32 decomposition against the FP64 oracle's at
    1e-5 (lambda relative, u normwise), stopping at the first near-tie (later
    components then follow a different deflation); then the FP64 steps given
    the GPU's own (lambda_hat, u_hat): lambda_hat = med_m <s^(m), s^(m)(u^3)>
    on the sketches deflated by the GPU's earlier components, and the final
    deflated sketches, both at 1e-12."""
    k = lam.shape[0]
    B = S_in.shape[0]
    compared = 0
    for c in range(k):
        if near_tie(ref.lam_tau[c]):
            print(f"{label}: component {c}: near-tie in the oracle's selection values, "
                  f"components {c}..{k - 1} not compared", flush=True)
            break
        el = abs(lam[c] - ref.lam[c]) / abs(ref.lam[c])
        eu = rel(U[c], ref.U[c])
        print(f"{label}: component {c}: lambda rel err {el:.2e}, u rel err {eu:.2e}", flush=True)
        assert el < 1e-5 and eu < 1e-5, (c, el, eu)
        compared += 1
    assert compared >= 1
    S = np.array(S_in, dtype=np.float64, copy=True)
    for c in range(k):
        lam_c = float(oracle.median(np.array([oracle.tuuu_sketch(S[m], h[m], xi[m], U[c]) for m in range(B)]),
                                   axis=0))
        assert abs(lam[c] - lam_c) <= 1e-12 * max(abs(lam_c), 1e-300), (c, lam[c], lam_c)
        for m in range(B):
            S[m] -= lam[c] * oracle.sketch_rank1_fft(U[c], U[c], U[c], h[m], xi[m], b)
    assert rel(S64_time, S) < 1e-12
    return compared


def test_decompose_fp32_full_size_c2(ctx):
    """n=200 FP32 dense, k=10, b=16384, B=10, L=50, T=30 batched: all ten
    components against the FP64 oracle (1e-5; near-ties reported, not failed),
    lambda_hat and the deflated sketches given the GPU's vectors (1e-12), and all
    ten against the planted truth."""
    n, k, b, B, L, T = 200, 10, 16384, 10, 50, 30
    P = planted_tensor(n, k, noise=0.05, seed=1, dtype=np.float32)
    tab, h, xi = _tables(ctx, 1, n, b, B)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    S_built = _time_sketch(ctx, tab, S64)
    u0 = np.stack([oracle.start_vectors_spec(1, c, L, n) for c in range(k)])
    lam, U, tau, flags = tsk.decompose(ctx, tab, S64, S32, k, L, T, dtype=tsk.F32,
                                       u0=torch.from_numpy(u0).to(DEV))
    lam, U = lam.cpu().numpy(), U.cpu().numpy()
    assert oracle.wrong_vectors(P.V, U) == 0
    # Theorem 1: each sketched estimate is off by O(||T||_F / sqrt(b)); allow 3x.
    tol = 3.0 * float(np.linalg.norm(P.T.astype(np.float64))) / np.sqrt(b)
    np.testing.assert_allclose(np.sort(lam), np.sort(P.lam), atol=tol)
    S_time = _oracle_sketches(P.T.astype(np.float64), h, xi, b)
    assert rel(S_built, S_time) < 1e-12
    ref = oracle.rtpm_sketched(S_time, h, xi, k, L, T, u0)
    n_cmp = check_fp32_decomposition(ref, lam, U, _time_sketch(ctx, tab, S64), S_built, h, xi, b, "C2")
    assert n_cmp == k, f"only {n_cmp} of {k} components compared (near-tie)"


def test_plain_path_equals_batched(ctx):
    n, k, b, B, L, T = 50, 3, 1024, 4, 6, 8
    P = planted_tensor(n, 3, noise=0.01, seed=5, dtype=np.float32)
    tab, h, xi = _tables(ctx, 2, n, b, B)
    # one build (its LDS atomics may add in any order), cloned for both paths
    S64_0, S32_0 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64_0, S32_0)
    out = []
    for plain in (False, True):
        S64, S32 = S64_0.clone(), S32_0.clone()
        r = tsk.decompose(ctx, tab, S64, S32, k, L, T, dtype=tsk.F32, seed=3, plain=plain)
        out.append([x.cpu().numpy() for x in r])
    for a, c in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, c)


def test_recreated_tables_do_not_replay_old_graphs(ctx):
    """Decompositions on tables created after others were destroyed (handles
    and sketch buffers may reuse addresses) match a fresh context's result."""
    n, k, L, T = 40, 2, 6, 6
    P = planted_tensor(n, 2, noise=0.01, seed=8, dtype=np.float32)
    Td = torch.from_numpy(P.T).to(DEV)
    results = {}
    for b, B in ((1024, 3), (2048, 4), (1024, 3)):
        h, xi = tsk.hash_generate(9, n, b, B)
        tab = tsk.Tables(ctx, h, xi, b)
        S64, S32 = tsk.new_sketch(tab, DEV)
        tsk.sketch_build_dense(ctx, tab, Td, S64, S32)
        lam, U, _, _ = tsk.decompose(ctx, tab, S64, S32, k, L, T, dtype=tsk.F64, seed=4)
        results.setdefault((b, B), []).append((lam.cpu().numpy(), U.cpu().numpy()))
        tab.close()
        del S64, S32
    c2 = tsk.Context(0)
    try:
        for (b, B), got in results.items():
            h, xi = tsk.hash_generate(9, n, b, B)
            tab = tsk.Tables(c2, h, xi, b)
            S64, S32 = tsk.new_sketch(tab, DEV)
            tsk.sketch_build_dense(c2, tab, Td, S64, S32)
            lam, U, _, _ = tsk.decompose(c2, tab, S64, S32, k, L, T, dtype=tsk.F64, seed=4)
            for lam_g, U_g in got:
                # FP64 builds add in any order: equal to rounding
                assert np.allclose(lam_g, lam.cpu().numpy(), rtol=1e-10, atol=0)
                assert np.allclose(U_g, U.cpu().numpy(), rtol=0, atol=1e-9)
            tab.close()
    finally:
        torch.cuda.synchronize()
        c2.close()


def test_graph_replay_is_stable(ctx):
    n, k, b, B, L, T = 64, 3, 4096, 5, 12, 10
    P = planted_tensor(n, 3, noise=0.02, seed=6, dtype=np.float32)
    tab, h, xi = _tables(ctx, 4, n, b, B)
    Td = torch.from_numpy(P.T).to(DEV)
    S64, S32 = tsk.new_sketch(tab, DEV)
    lam = torch.empty(k, dtype=torch.float64, device=DEV)
    U = torch.empty((k, n), dtype=torch.float64, device=DEV)
    tau = torch.empty(k, dtype=torch.int32, device=DEV)
    fl = torch.empty((k, L), dtype=torch.int32, device=DEV)
    S64_0, S32_0 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, Td, S64_0, S32_0)
    results = []
    for rep in range(4):
        S64.copy_(S64_0)
        S32.copy_(S32_0)
        tsk.decompose(ctx, tab, S64, S32, k, L, T, seed=7, lam_out=lam, U_out=U, tau_out=tau,
                      flags_out=fl)
        # eager work and a synchronisation between replays
        junk = torch.randn(1000, device=DEV).sum()
        torch.cuda.synchronize()
        results.append((lam.cpu().numpy().copy(), U.cpu().numpy().copy(), float(junk)))
    for r in results[1:]:
        np.testing.assert_array_equal(r[0], results[0][0])
        np.testing.assert_array_equal(r[1], results[0][1])
    plain = tsk.decompose(ctx, tab, *tsk.new_sketch(tab, DEV), k, L, T, seed=7, plain=True)
    del plain


def test_injective_hash_reduces_to_dense_power_method(ctx):
    n, b, B, k, L, T = 8, 512, 3, 3, 4, 12
    rng = np.random.default_rng(9)
    h = np.zeros((B, 3, n), dtype=np.uint32)
    h[:, 0] = np.arange(n)
    h[:, 1] = n * np.arange(n)
    h[:, 2] = n * n * np.arange(n)
    xi = rng.choice(np.array([-1, 1], dtype=np.int8), size=(B, 3, n))
    tab = tsk.Tables(ctx, h, xi, b)
    P = planted_tensor(n, k, noise=0.05, seed=3)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    u0 = np.stack([oracle.start_vectors_spec(4, c, L, n) for c in range(k)])
    lam, U, _, _ = tsk.decompose(ctx, tab, S64, S32, k, L, T, dtype=tsk.F64,
                                 u0=torch.from_numpy(u0).to(DEV))
    rd = oracle.rtpm_dense(P.T, k, L, T, u0)
    assert np.abs(lam.cpu().numpy() - rd.lam).max() < 1e-11
    assert np.abs(U.cpu().numpy() - rd.U).max() < 1e-11


def test_zero_tensor_sets_flags_and_stays_finite(ctx):
    n, b, B, k, L, T = 16, 256, 3, 2, 4, 3
    tab, _, _ = _tables(ctx, 3, n, b, B)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.zeros((n, n, n), dtype=torch.float32, device=DEV), S64, S32)
    lam, U, tau, flags = tsk.decompose(ctx, tab, S64, S32, k, L, T, seed=1)
    assert (flags.cpu().numpy() == 1).all()
    assert np.all(lam.cpu().numpy() == 0.0)
    Un = U.cpu().numpy()
    assert np.all(np.isfinite(Un))
    np.testing.assert_allclose(np.linalg.norm(Un, axis=1), 1.0, atol=1e-6)


def test_nan_input_is_flagged_not_propagated_into_u(ctx):
    n, b, B, L = 16, 256, 3, 4
    tab, _, _ = _tables(ctx, 3, n, b, B)
    T = torch.zeros((n, n, n), dtype=torch.float32, device=DEV)
    T[1, 2, 3] = float("nan")
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, T, S64, S32)
    U = torch.nn.functional.normalize(torch.randn((L, n), device=DEV), dim=1)
    flags = torch.zeros((L,), dtype=torch.int32, device=DEV)
    Uo = tsk.power_update(ctx, tab, U, S64=S64, S32=S32, flags=flags)
    assert (flags.cpu().numpy() == 1).all()
    np.testing.assert_array_equal(Uo.cpu().numpy(), U.cpu().numpy())


def test_argument_errors(ctx):
    h, xi = tsk.hash_generate(0, 10, 256, 2)
    with pytest.raises(tsk.TskError, match="EINVAL"):
        tsk.Tables(ctx, h, xi, 100)                  # b not a power of two
    with pytest.raises(tsk.TskError, match="EINVAL"):
        tsk.Tables(ctx, h, xi, 128)                  # h >= b
    h65, xi65 = tsk.hash_generate(0, 10, 256, 65)
    with pytest.raises(tsk.TskError, match="EINVAL"):
        tsk.Tables(ctx, h65, xi65, 256)              # B > 64
    hb, xb = tsk.hash_generate(0, 10, 131072, 2)
    with pytest.raises(tsk.TskError, match="EUNSUPPORTED"):
        tsk.Tables(ctx, hb, xb, 131072)
    hn, xn = tsk.hash_generate(0, 3000, 16384, 2)
    tabn = tsk.Tables(ctx, hn, xn, 16384)
    S64n, S32n = tsk.new_sketch(tabn, DEV)
    Un = torch.zeros((2, 3000), dtype=torch.float64, device=DEV)
    with pytest.raises(tsk.TskError, match="EUNSUPPORTED"):
        tsk.power_update(ctx, tabn, Un, S64=S64n, S32=S32n)   # n too large for LDS at this b
    h16, x16 = tsk.hash_generate(0, 10, 16384, 2)
    tab16 = tsk.Tables(ctx, h16, x16, 16384)
    S64, S32 = tsk.new_sketch(tab16, DEV)
    U32 = torch.zeros((2, 10), dtype=torch.float32, device=DEV)
    L = tsk.lib()
    st = L.tsk_power_update(ctx.handle, tab16.handle, 0, S64.data_ptr(), S32.data_ptr(), 2,
                            U32.data_ptr(), U32.data_ptr(), None, None, None)
    assert st == -1                                            # aliasing in/out
    with pytest.raises(tsk.TskError, match="EINVAL"):
        tsk.decompose(ctx, tab16, S64, S32, 11, 2, 2)          # k > n


@pytest.mark.parametrize("B", [1, 2, 3, 4, 15, 16, 17, 20, 31, 32, 33, 40, 63, 64, 65, 80])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_median_normalize_matches_oracle(ctx, B, dtype):
    """Median over sketches and normalisation (Algorithm 1) on given estimates:
    values from a small set (many ties), a NaN coordinate, an all-zero restart
    (fallback and flag), n across one and several coordinates per thread."""
    print(f"median B={B} {dtype}", flush=True)
    rng = np.random.default_rng(B)
    for n in (1, 7, 300, 1500):
        L = 4
        V = rng.integers(-3, 4, size=(L, B, n)).astype(np.float64) * 0.25
        V[1] += rng.standard_normal((B, n)) * 1e-3            # mostly distinct
        if n > 3:
            V[2, rng.integers(0, B), 3] = np.nan                 # NaN -> NaN coordinate -> fallback
        V[3] = 0.0                                               # zero median -> fallback
        U_in = rng.standard_normal((L, n))
        if dtype == torch.float32:
            V = V.astype(np.float32).astype(np.float64)
            U_in = U_in.astype(np.float32).astype(np.float64)
        Vd = torch.from_numpy(V).to(device=DEV, dtype=dtype)
        Ud = torch.from_numpy(U_in).to(device=DEV, dtype=dtype)
        flags = torch.zeros(L, dtype=torch.int32, device=DEV)
        out = tsk.median_normalize(ctx, Vd, Ud, flags=flags).cpu().numpy()
        vbar = oracle.contract.median(V, axis=1)
        tol = 1e-6 if dtype == torch.float32 else 1e-14
        for tau in range(L):
            nrm = np.linalg.norm(vbar[tau])
            if nrm > 0 and np.isfinite(nrm):
                assert flags[tau].item() == 0
                np.testing.assert_allclose(out[tau], vbar[tau] / nrm, rtol=0, atol=tol)
            else:
                assert flags[tau].item() == 1
                np.testing.assert_array_equal(out[tau], U_in[tau])


@pytest.mark.parametrize("B", [1, 64])
def test_decompose_at_one_and_the_most_sketches(ctx, B):
    """B = 1 (the median is the single estimate) and B = 64 (the most a table
    set holds: every lane of a wave carries a value in the medians of the
    selection and deflation): the whole of Algorithm 1 in FP64 against the
    oracle."""
    print(f"decompose B={B}", flush=True)
    n, k, b, L, T = 30, 2, 512, 3, 4
    P = planted_tensor(n, 2, noise=0.01, seed=13)
    tab, h, xi = _tables(ctx, 14, n, b, B)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    u0 = np.stack([oracle.start_vectors_spec(5, c, L, n) for c in range(k)])
    lam, U, tau, flags = tsk.decompose(ctx, tab, S64, S32, k, L, T, dtype=tsk.F64,
                                       u0=torch.from_numpy(u0).to(DEV))
    ref = oracle.rtpm_sketched(_oracle_sketches(P.T, h, xi, b), h, xi, k, L, T, u0)
    assert rel(lam.cpu().numpy(), ref.lam) < 1e-12
    assert rel(U.cpu().numpy(), ref.U) < 1e-12
    np.testing.assert_array_equal(tau.cpu().numpy(), ref.tau)


@pytest.mark.parametrize("B,dtype,T,tol", [(20, tsk.F64, 6, 1e-12), (40, tsk.F32, 25, 1e-5)])
def test_decompose_with_separate_median_launch(ctx, B, dtype, T, tol):
    """B > 16: the median of each step is a launch of its own inside the graph
    (not the power kernel's prologue); whole of Algorithm 1 against the oracle."""
    print(f"decompose separate median B={B}", flush=True)
    n, k, b, L = 30, 2, 512, 5
    P = planted_tensor(n, 2, noise=0.01, seed=11)
    tab, h, xi = _tables(ctx, 12, n, b, B)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    S_built = _time_sketch(ctx, tab, S64)
    u0 = np.stack([oracle.start_vectors_spec(3, c, L, n) for c in range(k)])
    if dtype == tsk.F32:
        u0 = u0.astype(np.float32).astype(np.float64)
    lam, U, tau, flags = tsk.decompose(ctx, tab, S64, S32, k, L, T, dtype=dtype,
                                       u0=torch.from_numpy(u0).to(DEV))
    S_time = _oracle_sketches(P.T, h, xi, b)
    if dtype == tsk.F64:
        ref = oracle.rtpm_sketched(S_time, h, xi, k, L, T, u0)
        assert rel(lam.cpu().numpy(), ref.lam) < tol
        assert rel(U.cpu().numpy(), ref.U) < tol
        np.testing.assert_array_equal(flags.cpu().numpy(), ref.flags)
    else:
        # FP32 steps: every component at 1e-5 (near-ties reported), FP64 steps at 1e-12
        ref = oracle.rtpm_sketched(S_time, h, xi, k, L, T, u0)
        n_cmp = check_fp32_decomposition(ref, lam.cpu().numpy(), U.cpu().numpy(),
                                         _time_sketch(ctx, tab, S64), S_built, h, xi, b,
                                         f"separate median B={B}")
        assert n_cmp == k
