"""Sketch lengths beyond one work-group's LDS (b = 32768 and 65536): the split
transforms (residue sub-transforms recombined in global memory) and the
bucket-range split of the dense build, against numpy.fft and the oracle.

Bars: FP64 within 1e-12 normwise relative, FP32 within 1e-5.
"""
import numpy as np
import pytest

import oracle
from oracle import gradients as G
from paper_1506_04448_amd.workloads import planted_tensor, factor_instances

torch = pytest.importorskip("torch")
import paper_1506_04448_amd as tsk  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rel(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm(ref)
    return np.linalg.norm(a - ref) / (d if d > 0 else 1.0)


@pytest.fixture(scope="module")
def ctx():
    c = tsk.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("b", [32768, 65536])
def test_split_spectrum_roundtrip_and_numpy(ctx, b):
    print(f"large spectra b={b}", flush=True)
    B = 3
    rng = np.random.default_rng(b)
    s = rng.standard_normal((B, b))
    S64 = torch.zeros((B, b // 2 + 1, 2), dtype=torch.float64, device=DEV)
    S32 = torch.zeros((B, b // 2 + 1, 2), dtype=torch.float32, device=DEV)
    tsk.sketch_from_time(ctx, torch.from_numpy(s).to(DEV), S64, S32)
    ref = np.fft.rfft(s, axis=1)
    got = S64.cpu().numpy()
    assert rel(got[..., 0] + 1j * got[..., 1], ref) < 1e-13
    back = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    assert rel(back, s) < 1e-13
    np.testing.assert_array_equal(S32.cpu().numpy(), got.astype(np.float32))


@pytest.mark.parametrize("b,dt", [(32768, np.float64), (65536, np.float32)])
def test_split_dense_build(ctx, b, dt):
    print(f"large build b={b}", flush=True)
    n, B = 30, 3
    P = planted_tensor(n, 3, noise=0.05, seed=2, dtype=dt)
    h, xi = tsk.hash_generate(4, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    got = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    tol = 1e-12 if dt == np.float64 else 1e-5
    for m in range(B):
        ref = oracle.sketch_dense(P.T.astype(np.float64), h[m], xi[m], b)
        assert rel(got[m], ref) < tol


@pytest.mark.parametrize("b,dt,n,mode", [(65536, np.float32, 300, "clustered"),
                                         (32768, np.float64, 260, "clustered"),
                                         (65536, np.float64, 130, "uniform"),
                                         (32768, np.float32, 67, "uniform"),
                                         (65536, np.float32, 1, "uniform")])
def test_bucket_range_build_of_integer_tensor_is_exact(ctx, b, dt, n, mode):
    """Sketches longer than one work-group's 16384 buckets: each work-group
    owns one range of buckets and keeps the entries that land in it.  Small
    integer entries make every bucket sum exact on both sides.  With h3
    clustered around zero ([b - 20, b) and [0, 20)) a fibre's entries all fall
    in one or two ranges, on both sides of the wrap from bucket b - 1 to 0."""
    print(f"range build b={b} n={n} {mode} {np.dtype(dt).name}", flush=True)
    rng = np.random.default_rng(n + b)
    T = rng.integers(-7, 8, size=(n, n, n)).astype(dt)
    B = 2
    h, xi = tsk.hash_generate(31 + n, n, b, B)
    if mode == "clustered":
        near = rng.integers(-20, 20, size=(B, n))
        h[:, 2, :] = (near % b).astype(np.uint32)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    Td = torch.from_numpy(T).to(DEV)
    tsk.sketch_build_dense(ctx, tab, Td, S64, S32)
    got = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    ref = np.stack([oracle.sketch_dense(T.astype(np.float64), h[m], xi[m], b) for m in range(B)])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9)
    S64b, S32b = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, Td, S64b, S32b)
    np.testing.assert_array_equal(S64b.cpu().numpy(), S64.cpu().numpy())
    tab.close()


def _buckets_by_definition(Tdev, h, xi, b, ts):
    """s(t) of Eq. (1) for the buckets ts, one by one: the entries (i, j, k)
    with h1(i) + h2(j) + h3(k) = t mod b, read from the device tensor."""
    n = Tdev.shape[0]
    h1, h2, h3 = (h[j].astype(np.int64) for j in range(3))
    order = np.argsort(h3, kind="stable")
    hs = h3[order]
    c = (h1[:, None] + h2[None, :]) % b
    out = []
    flat = Tdev.reshape(-1)
    for t in ts:
        v = (t - c) % b
        lo = np.searchsorted(hs, v, side="left").ravel()
        hi = np.searchsorted(hs, v, side="right").ravel()
        cnt = hi - lo
        pair = np.repeat(np.arange(n * n), cnt)
        first = np.repeat(lo, cnt)
        offs = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        k = order[first + offs]
        i, j = pair // n, pair % n
        idx = torch.from_numpy(i * n * n + j * n + k).to(Tdev.device)
        vals = flat[idx].double().cpu().numpy()
        sg = xi[0][i].astype(np.float64) * xi[1][j] * xi[2][k]
        out.append(float(np.sum(sg * vals)))
    return np.array(out)


def test_bucket_range_build_full_size_sampled(ctx):
    """The differentiation workload's build shape (n = 1000, FP32, b = 65536,
    four ranges per sketch) at full size: 48 sampled buckets per sketch
    against Eq. (1) summed bucket by bucket in FP64."""
    from paper_1506_04448_amd.workloads import planted_tensor_device
    n, b, B = 1000, 65536, 2
    print(f"range build full size n={n} b={b}", flush=True)
    X = planted_tensor_device(n, 100, 0.1, seed=3, device=DEV)
    Tdev = X.T
    h, xi = tsk.hash_generate(77, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, Tdev, S64, S32)
    got = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    rng = np.random.default_rng(5)
    for m in range(B):
        ts = np.concatenate([[0, 16383, 16384, 32767, 32768, 49151, 49152, 65535],
                             rng.integers(0, b, size=40)])
        ref = _buckets_by_definition(Tdev, h[m], xi[m], b, ts)
        assert rel(got[m][ts], ref) < 1e-5, (m, rel(got[m][ts], ref))
    tab.close()


@pytest.mark.parametrize("b", [32768, 65536])
def test_split_factor_build_and_deflate(ctx, b):
    print(f"large factors b={b}", flush=True)
    inst = factor_instances(1, seed=8, n_range=(60, 60), k_range=(4, 4), b_choices=(b,))[0]
    B = 2
    h, xi = tsk.hash_generate(5, inst.n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_factors(ctx, tab, torch.from_numpy(inst.lam).to(DEV), torch.from_numpy(inst.A).to(DEV),
                             S64, S32)
    got = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    for m in range(B):
        ref = oracle.sketch_factors(inst.lam, inst.A, h[m], xi[m], b)
        assert rel(got[m], ref) < 1e-12
    # deflating the first two components leaves the sketch of the other two
    tsk.sketch_deflate(ctx, tab, torch.from_numpy(inst.lam[:2]).to(DEV), torch.from_numpy(inst.A[:2]).to(DEV),
                       S64, S32)
    got = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    for m in range(B):
        ref = oracle.sketch_factors(inst.lam[2:], inst.A[2:], h[m], xi[m], b)
        assert rel(got[m], ref) < 1e-12


# n = 1024 and 1025 at b = 65536 sit on both sides of the bound below which the
# inverse sub-transforms leave out their last two passes.
@pytest.mark.parametrize("b,n", [(32768, 200), (65536, 200), (65536, 1024), (65536, 1025)])
def test_large_power_update_and_uuu(ctx, b, n):
    print(f"large power b={b} n={n}", flush=True)
    B, L = 4, 3
    rng = np.random.default_rng(b + 1)
    h, xi = tsk.hash_generate(6, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S_time = rng.standard_normal((B, b))
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_from_time(ctx, torch.from_numpy(S_time).to(DEV), S64, S32)
    U = rng.standard_normal((L, n))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    Ud = torch.from_numpy(U.astype(np.float32)).to(DEV)
    V = tsk.contract_tiuu(ctx, tab, Ud, S32=S32).cpu().numpy()
    Uf = U.astype(np.float32).astype(np.float64)
    for m in range(B):
        ref = oracle.power_update_sketch(S_time[m], h[m], xi[m], Uf)
        assert rel(V[:, m], ref) < 1e-5
    Vo, Unew, _ = oracle.power_update(S_time, h, xi, Uf)
    got = tsk.power_update(ctx, tab, Ud, S32=S32).cpu().numpy()
    assert rel(got, Unew) < 1e-5
    lam_med, lam_per = tsk.contract_uuu(ctx, tab, Ud, S32=S32)
    rper, rmed = oracle.contract_uuu(S_time, h, xi, Uf)
    assert rel(lam_per.cpu().numpy(), rper) < 1e-5
    assert rel(lam_med.cpu().numpy(), rmed) < 1e-5
    # the three mode read-offs (gradient of T(u,u,u))
    f_med, f_per, grad = tsk.contract_tuuu_grad(ctx, tab, Ud, S32=S32)
    _, _, rgrad = G.tuuu_with_grad(S_time, h, xi, Uf)
    assert rel(grad.cpu().numpy(), rgrad) < 1e-5


@pytest.mark.parametrize("B", [4, 20])
def test_large_decompose_fp32_matches_oracle(ctx, B):
    """B = 4: the median of each step is the split kernel's prologue; B = 20:
    it runs as a launch of its own before the step."""
    print(f"large decompose b=65536 B={B}", flush=True)
    n, k, b, L, T = 80, 3, 65536, 6, 8
    P = planted_tensor(n, k, noise=0.02, seed=9, lam_range=(1.0, 3.0))
    h, xi = tsk.hash_generate(9, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    lam, U, tau, fl = tsk.decompose(ctx, tab, S64, S32, k, L, T, dtype=tsk.F32, seed=9)
    S_time = np.stack([oracle.sketch_dense(P.T, h[m], xi[m], b) for m in range(B)])
    u0 = np.stack([oracle.start_vectors_spec(9, c, L, n) for c in range(k)])
    r = oracle.rtpm_sketched(S_time, h, xi, k, L, T, u0)
    lam = lam.cpu().numpy()
    U = U.cpu().numpy()
    assert abs(lam[0] - r.lam[0]) <= 1e-5 * abs(r.lam[0])
    assert rel(U[0], r.U[0]) < 1e-5
    # planted components are recovered
    assert oracle.wrong_vectors(P.V, U) == 0


def test_split_step_single_sketch_single_vector(ctx):
    """The smallest split-step launch (b = 65536, B = 1, L = 1, n = 5): one
    work-group, the median of one estimate, against the oracle."""
    n, b = 5, 65536
    rng = np.random.default_rng(23)
    h, xi = tsk.hash_generate(23, n, b, 1)
    tab = tsk.Tables(ctx, h, xi, b)
    S_time = rng.standard_normal((1, b))
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_from_time(ctx, torch.from_numpy(S_time).to(DEV), S64, S32)
    U = rng.standard_normal((1, n))
    U /= np.linalg.norm(U)
    Uf = U.astype(np.float32).astype(np.float64)
    got = tsk.power_update(ctx, tab, torch.from_numpy(U.astype(np.float32)).to(DEV), S32=S32).cpu().numpy()
    _, Unew, _ = oracle.power_update(S_time, h, xi, Uf)
    assert rel(got, Unew) < 1e-5
    tab.close()


def test_large_decompose_with_u_beyond_lds(ctx):
    """n = 6000: u no longer fits the LDS beside the split kernel's buffer, so
    the count sketches read it from global memory and the median of each step
    is a launch of its own.  Factor sketch of two unit vectors; the first
    component against the oracle's Algorithm 1 on the same sketch."""
    print("large decompose b=65536 n=6000", flush=True)
    n, b, B, L, T = 6000, 65536, 2, 2, 3
    rng = np.random.default_rng(17)
    A = rng.standard_normal((2, n))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    lamf = np.array([3.0, 1.5])
    h, xi = tsk.hash_generate(17, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_factors(ctx, tab, torch.from_numpy(lamf).to(DEV), torch.from_numpy(A).to(DEV), S64, S32)
    S_time = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    lam, U, _, _ = tsk.decompose(ctx, tab, S64, S32, 1, L, T, dtype=tsk.F32, seed=17)
    u0 = np.stack([oracle.start_vectors_spec(17, 0, L, n)])
    r = oracle.rtpm_sketched(S_time, h, xi, 1, L, T, u0)
    assert abs(float(lam.cpu().numpy()[0]) - r.lam[0]) <= 1e-5 * abs(r.lam[0])
    assert rel(U.cpu().numpy()[0], r.U[0]) < 1e-5
    tab.close()


def test_large_cp_loss_fp32(ctx):
    print("large cp loss b=65536", flush=True)
    n, b, B, k = 40, 65536, 2, 3
    rng = np.random.default_rng(11)
    h, xi = tsk.hash_generate(11, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S_time = rng.standard_normal((B, b))
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_from_time(ctx, torch.from_numpy(S_time).to(DEV), S64, S32)
    lam = rng.uniform(0.5, 2.0, k).astype(np.float32)
    U = rng.standard_normal((k, n)).astype(np.float32)
    loss, g_lam, g_U = tsk.cp_loss(ctx, tab, S64, torch.from_numpy(lam).to(DEV), torch.from_numpy(U).to(DEV))
    rloss, rg_lam, rg_U = G.cp_loss_grad(S_time, h, xi, lam.astype(np.float64), U.astype(np.float64))
    assert abs(float(loss) - rloss) <= 1e-10 * rloss
    assert rel(g_lam.cpu().numpy(), rg_lam) < 1e-5
    assert rel(g_U.cpu().numpy(), rg_U) < 1e-5


def test_large_unsupported_paths(ctx):
    h, xi = tsk.hash_generate(1, 10, 32768, 2)
    tab = tsk.Tables(ctx, h, xi, 32768)
    S64, S32 = tsk.new_sketch(tab, DEV)
    U = torch.zeros((2, 10), dtype=torch.float64, device=DEV)
    with pytest.raises(tsk.TskError, match="EUNSUPPORTED"):
        tsk.contract_uuu(ctx, tab, U, S64=S64)
    W = torch.zeros((5, 10), dtype=torch.float32, device=DEV)
    z = torch.zeros(1, dtype=torch.int32, device=DEV)
    with pytest.raises(tsk.TskError, match="EUNSUPPORTED"):
        tsk.sketch_build_docs(ctx, tab, torch.zeros(2, dtype=torch.int32, device=DEV), z, z, 5, W, 1.0, S64, S32)
