"""The allocation-free power step against tsk_power_update, through the C ABI.

Both run the same kernels on the same inputs, so the results must agree bit
for bit.  Each case starts on a fresh context, so the allocation-free call runs
before any other call could have made its workspaces: a path that would
allocate fails there with TSK_EUNSUPPORTED.  Two calls in a row share the
library's static scratch array; the second takes fewer vectors.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_1506_04448_amd as tsk  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _unit_rows(rng, L, n, dtype):
    U = rng.standard_normal((L, n))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    return torch.from_numpy(U).to(device=DEV, dtype=dtype)


# (n, b, B, L first call, L second call, dtype): the dense benchmark's shape,
# an FP64 case, the split transforms at b = 65536 and a median run as its own
# launch (n beyond what the power kernel's prologue stages).
CASES = [
    (200, 16384, 10, 50, 7, torch.float32),
    (50, 1024, 4, 10, 3, torch.float64),
    (200, 65536, 4, 3, 1, torch.float32),
    (2000, 4096, 8, 5, 2, torch.float32),
]


@pytest.mark.parametrize("n,b,B,L1,L2,dtype", CASES)
def test_noalloc_power_step_equals_power_update(n, b, B, L1, L2, dtype):
    print(f"noalloc n={n} b={b} B={B} L={L1},{L2} {dtype}", flush=True)
    ctx = tsk.Context(0)
    h, xi = tsk.hash_generate(11, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    rng = np.random.default_rng(n + b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_from_time(ctx, torch.from_numpy(rng.standard_normal((B, b))).to(DEV), S64, S32)
    spec = dict(S64=S64) if dtype == torch.float64 else dict(S32=S32)
    results = []
    for L in (L1, L2):
        U = _unit_rows(rng, L, n, dtype)
        out = torch.full((L, n), float("nan"), dtype=dtype, device=DEV)
        fl = torch.zeros((L,), dtype=torch.int32, device=DEV)
        tsk.power_update_noalloc(ctx, tab, U, out, flags=fl, **spec)
        results.append((U, out, fl))
    torch.cuda.synchronize()
    for U, out, fl in results:
        L = U.shape[0]
        fl_ref = torch.zeros((L,), dtype=torch.int32, device=DEV)
        ref = tsk.power_update(ctx, tab, U, flags=fl_ref, **spec)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (L, (out - ref).abs().max().item())
        assert torch.equal(fl, fl_ref)
    tab.close()
    ctx.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    ctx = tsk.Context(0)
    n, b, B, L = 100, 65536, 16, 8   # the split buffers alone take 96 MiB
    h, xi = tsk.hash_generate(12, n, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    U = torch.zeros((L, n), dtype=torch.float32, device=DEV)
    out = torch.zeros_like(U)
    with pytest.raises(tsk.TskError) as e:
        tsk.power_update_noalloc(ctx, tab, U, out, S32=S32)
    assert e.value.status == -1 and "scratch" in str(e.value)
    tab.close()
    ctx.close()
