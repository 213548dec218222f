"""Parity of the gradient extensions (HIP path through the C ABI) with the CPU
oracle: the T(u,u,u) estimate with its gradient, the sketched CP loss with its
gradients, the autograd wrappers and the Adam refinement.

Bars: FP64 within 1e-12 normwise relative, FP32 within 1e-5 normwise relative.
Inputs: seeded random time-domain sketches and vectors (a gradient is defined
for any sketch), planted tensors for the refinement.
"""
import numpy as np
import pytest

import oracle
from oracle import gradients as G
from paper_1506_04448_amd.workloads import planted_tensor

torch = pytest.importorskip("torch")
import paper_1506_04448_amd as tsk  # noqa: E402
from paper_1506_04448_amd import autograd as tag  # noqa: E402

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


def _setup(ctx, seed, n, b, B):
    h, xi = tsk.hash_generate(seed, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    rng = np.random.default_rng(seed)
    S_time = rng.standard_normal((B, b))
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_from_time(ctx, torch.from_numpy(S_time).to(DEV), S64, S32)
    return tab, h, xi, S_time, S64, S32, rng


@pytest.mark.parametrize("n,b,B,L,dt", [(37, 1024, 5, 6, np.float64), (37, 1024, 4, 6, np.float64),
                                        (200, 16384, 10, 8, np.float32), (123, 4096, 3, 5, np.float32),
                                        (1, 64, 1, 2, np.float64), (50, 256, 64, 3, np.float64)])
def test_tuuu_grad_matches_oracle(ctx, n, b, B, L, dt):
    print(f"tuuu_grad n={n} b={b} B={B} L={L} {np.dtype(dt).name}", flush=True)
    tab, h, xi, S_time, S64, S32, rng = _setup(ctx, 21 + n, n, b, B)
    U = rng.standard_normal((L, n))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    U = U.astype(dt)
    Ud = torch.from_numpy(U).to(DEV)
    scale = rng.uniform(0.5, 2.0, L).astype(dt)
    f_med, f_per, grad = tsk.contract_tuuu_grad(ctx, tab, Ud, S64=S64, S32=S32,
                                                scale=torch.from_numpy(scale).to(DEV))
    rf_med, rf_per, rgrad = G.tuuu_with_grad(S_time, h, xi, U.astype(np.float64))
    tol = 1e-12 if dt == np.float64 else 1e-5
    assert rel(f_per.cpu().numpy(), rf_per) < tol
    assert rel(f_med.cpu().numpy(), rf_med) < tol
    g = grad.cpu().numpy()
    for tau in range(L):
        assert rel(g[tau], scale[tau] * rgrad[tau]) < tol, (tau, rel(g[tau], scale[tau] * rgrad[tau]))


@pytest.mark.parametrize("n,b,B,k,dt", [(30, 512, 3, 4, np.float64), (30, 512, 4, 4, np.float32),
                                        (100, 4096, 8, 10, np.float32), (64, 16384, 2, 3, np.float64)])
def test_cp_loss_matches_oracle(ctx, n, b, B, k, dt):
    print(f"cp_loss n={n} b={b} B={B} k={k} {np.dtype(dt).name}", flush=True)
    tab, h, xi, S_time, S64, S32, rng = _setup(ctx, 40 + n, n, b, B)
    lam = rng.uniform(0.5, 2.0, k).astype(dt)
    U = rng.standard_normal((k, n))
    U = (U / np.linalg.norm(U, axis=1, keepdims=True)).astype(dt)
    loss, g_lam, g_U = tsk.cp_loss(ctx, tab, S64, torch.from_numpy(lam).to(DEV),
                                   torch.from_numpy(U).to(DEV))
    rloss, rg_lam, rg_U = G.cp_loss_grad(S_time, h, xi, lam.astype(np.float64), U.astype(np.float64))
    tol = 1e-12 if dt == np.float64 else 1e-5
    assert abs(float(loss) - rloss) <= tol * abs(rloss)
    assert rel(g_lam.cpu().numpy(), rg_lam) < tol
    assert rel(g_U.cpu().numpy(), rg_U) < tol
    # loss only, and a scale on the gradients
    loss2, a, c = tsk.cp_loss(ctx, tab, S64, torch.from_numpy(lam).to(DEV),
                              torch.from_numpy(U).to(DEV), grads=False)
    assert a is None and c is None and float(loss2) == float(loss)
    sc = torch.tensor([-3.0], dtype=torch.from_numpy(lam).dtype, device=DEV)
    _, g_lam3, g_U3 = tsk.cp_loss(ctx, tab, S64, torch.from_numpy(lam).to(DEV),
                                  torch.from_numpy(U).to(DEV), scale=sc)
    assert rel(g_lam3.cpu().numpy(), -3.0 * rg_lam) < tol
    assert rel(g_U3.cpu().numpy(), -3.0 * rg_U) < tol


def test_cp_loss_injective_hash_equals_dense_loss(ctx):
    n, b, B, k = 8, 512, 2, 3
    rng = np.random.default_rng(12)
    P = planted_tensor(n, 3, noise=0.1, seed=12)
    h = np.zeros((B, 3, n), dtype=np.uint32)
    h[:, 0] = np.arange(n)
    h[:, 1] = n * np.arange(n)
    h[:, 2] = n * n * np.arange(n)
    xi = rng.choice(np.array([-1, 1], dtype=np.int8), size=(B, 3, n))
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    lam = rng.uniform(0.5, 2.0, k)
    U = rng.standard_normal((k, n))
    loss, g_lam, g_U = tsk.cp_loss(ctx, tab, S64, torch.from_numpy(lam).to(DEV),
                                   torch.from_numpy(U).to(DEV))
    R = P.T - np.einsum("r,ri,rj,rk->ijk", lam, U, U, U)
    assert abs(float(loss) - np.sum(R * R)) <= 1e-12 * np.sum(R * R)
    dense_gU = -6.0 * lam[:, None] * np.einsum("ijk,rj,rk->ri", R, U, U)
    assert rel(g_U.cpu().numpy(), dense_gU) < 1e-12
    assert rel(g_lam.cpu().numpy(), -2.0 * np.einsum("ijk,ri,rj,rk->r", R, U, U, U)) < 1e-12


def test_autograd_functions_gradcheck_and_oracle(ctx):
    n, b, B, k, L = 12, 256, 3, 2, 3
    tab, h, xi, S_time, S64, S32, rng = _setup(ctx, 77, n, b, B)
    sk = tag.SketchHandle(ctx, tab, S64, S32)
    lam = torch.tensor(rng.uniform(0.5, 2.0, k), device=DEV, requires_grad=True)
    U = torch.tensor(rng.standard_normal((k, n)), device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, c: tag.sketched_cp_loss(a, c, sk), (lam, U),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)
    Uv = torch.tensor(rng.standard_normal((L, n)), device=DEV, requires_grad=True)
    assert torch.autograd.gradcheck(lambda c: tag.tuuu(c, sk), (Uv,), eps=1e-6, atol=1e-6, rtol=1e-5)
    # the CP loss's backward is its gradient times the upstream gradient
    c = 0.37
    lam.grad = None
    U.grad = None
    (c * tag.sketched_cp_loss(lam, U, sk)).backward()
    _, rg_lam, rg_U = G.cp_loss_grad(S_time, h, xi, lam.detach().cpu().numpy(), U.detach().cpu().numpy())
    assert rel(lam.grad.cpu().numpy(), c * rg_lam) < 1e-12
    assert rel(U.grad.cpu().numpy(), c * rg_U) < 1e-12
    # no gradient wanted: the forward returns the loss alone
    with torch.no_grad():
        l0 = tag.sketched_cp_loss(lam, U, sk)
    assert abs(float(l0) - G.cp_loss(S_time, h, xi, lam.detach().cpu().numpy(), U.detach().cpu().numpy())) \
        <= 1e-12 * abs(float(l0))
    # the backward pass equals the oracle gradient with the upstream weights
    w = torch.tensor(rng.standard_normal(L), device=DEV)
    (tag.tuuu(Uv, sk) * w).sum().backward()
    _, _, rgrad = G.tuuu_with_grad(S_time, h, xi, Uv.detach().cpu().numpy())
    assert rel(Uv.grad.cpu().numpy(), w.cpu().numpy()[:, None] * rgrad) < 1e-12


def test_adam_refinement_lowers_sketched_and_dense_loss(ctx):
    n, k, b, B, L, T = 60, 4, 4096, 8, 10, 15
    P = planted_tensor(n, k, noise=0.05, seed=5, dtype=np.float32)
    h, xi = tsk.hash_generate(5, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    Td = torch.from_numpy(P.T).to(DEV)
    tsk.sketch_build_dense(ctx, tab, Td, S64, S32)
    S64_0 = S64.clone()
    lam, U, _, _ = tsk.decompose(ctx, tab, S64, S32, k, L, T, dtype=tsk.F32, seed=5)
    sk = tag.SketchHandle(ctx, tab, S64_0, None)
    lam_r, U_r, losses = tag.refine_adam(sk, lam, U, steps=60, lr=2e-3)
    losses = losses.cpu().numpy()
    assert np.all(np.isfinite(losses))
    assert losses[-1] < losses[0]
    # oracle check of the final sketched loss
    S_time = np.stack([oracle.sketch_dense(P.T.astype(np.float64), h[m], xi[m], b) for m in range(B)])
    rl = G.cp_loss(S_time, h, xi, lam_r.double().cpu().numpy(), U_r.double().cpu().numpy())
    assert abs(losses[-1] - rl) <= 1e-4 * rl
    # fitting the sketches does not move far from the tensor itself
    def dense_res(lm, Um):
        R = P.T.astype(np.float64) - np.einsum("r,ri,rj,rk->ijk", lm, Um, Um, Um)
        return float(np.sum(R * R))
    assert dense_res(lam_r.double().cpu().numpy(), U_r.double().cpu().numpy()) <= \
        1.5 * dense_res(lam.cpu().numpy(), U.cpu().numpy())


def test_cp_gradient_fp32_at_c5_sketch_size_agrees_with_dense_fp64(ctx):
    """The differentiation workload's check instance: n = 100, k = 10 planted
    tensor with noise 0.1, random hashes, B = 16 sketches of b = 65536, FP32
    vectors.  The sketched gradients estimate the dense FP64 CP-loss gradients
    without bias with an error that falls as 1/sqrt(b) (about 8/sqrt(b) for U
    and 3/sqrt(b) for lam on the CPU oracle across hash seeds); the bars are
    twice that.  The FP32 result also matches the oracle's FP64 sketched
    gradient on the same sketches at the FP32 bar."""
    n, k, b, B = 100, 10, 65536, 16
    print(f"cp grad vs dense n={n} k={k} b={b} B={B}", flush=True)
    P = planted_tensor(n, k, noise=0.1, seed=5)
    rng = np.random.default_rng(5)
    lam = P.lam * (1.0 + 0.05 * rng.standard_normal(k))
    U = P.V + 0.02 * rng.standard_normal(P.V.shape)
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    lam32, U32 = lam.astype(np.float32), U.astype(np.float32)
    h, xi = tsk.hash_generate(105, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    loss, g_lam, g_U = tsk.cp_loss(ctx, tab, S64, torch.from_numpy(lam32).to(DEV),
                                   torch.from_numpy(U32).to(DEV))
    l64, u64 = lam32.astype(np.float64), U32.astype(np.float64)
    R = P.T - np.einsum("r,ri,rj,rk->ijk", l64, u64, u64, u64)
    d_lam = -2.0 * np.einsum("ijk,ri,rj,rk->r", R, u64, u64, u64)
    d_U = -6.0 * l64[:, None] * np.einsum("ijk,rj,rk->ri", R, u64, u64)
    assert abs(float(loss) - np.sum(R * R)) / np.sum(R * R) < 2.0 / np.sqrt(b)
    assert rel(g_lam.cpu().numpy(), d_lam) < 2.0 * 3.0 / np.sqrt(b)
    assert rel(g_U.cpu().numpy(), d_U) < 2.0 * 8.0 / np.sqrt(b)
    S_time = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    rloss, rg_lam, rg_U = G.cp_loss_grad(S_time, h, xi, l64, u64)
    assert abs(float(loss) - rloss) <= 1e-5 * abs(rloss)
    assert rel(g_lam.cpu().numpy(), rg_lam) < 1e-5
    assert rel(g_U.cpu().numpy(), rg_U) < 1e-5
    tab.close()
