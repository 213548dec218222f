"""Batched decomposition of uneven instances (one HIP graph with parallel
branches) against the same instances decomposed one by one, and the FP64
instance against the oracle.

Bar: bit-identical to the one-by-one results (the same kernels run on the same
inputs; only their placement on the device differs); FP64 within 1e-12 of the
oracle.  Inputs: factor instances (tensor never formed), seeded.
"""
import numpy as np
import pytest

import oracle
from paper_1506_04448_amd.workloads import factor_instances

torch = pytest.importorskip("torch")
import paper_1506_04448_amd as tsk  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# (n, k, b, B, dtype, L, T)
SHAPES = [(40, 3, 1024, 4, tsk.F64, 6, 10), (150, 6, 4096, 8, tsk.F32, 12, 8),
          (90, 4, 16384, 5, tsk.F32, 10, 6), (300, 5, 4096, 3, tsk.F32, 7, 9),
          (25, 2, 256, 6, tsk.F64, 5, 12), (1000, 7, 16384, 8, tsk.F32, 16, 5),
          # the split transforms of b = 65536, as in the batched workload
          (700, 4, 65536, 8, tsk.F32, 6, 4)]


@pytest.fixture(scope="module")
def ctx():
    c = tsk.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _instances(ctx):
    out = []
    for i, (n, k, b, B, dt, L, T) in enumerate(SHAPES):
        inst = factor_instances(1, seed=100 + i, n_range=(n, n), k_range=(k, k), b_choices=(b,))[0]
        h, xi = tsk.hash_generate(200 + i, n, b, B)
        tab = tsk.Tables(ctx, h, xi, b)
        S64, S32 = tsk.new_sketch(tab, DEV)
        tsk.sketch_build_factors(ctx, tab, torch.from_numpy(inst.lam).to(DEV),
                                 torch.from_numpy(inst.A).to(DEV), S64, S32)
        out.append(dict(inst=inst, h=h, xi=xi, tab=tab, S64=S64, S32=S32, dt=dt, L=L, T=T, k=k))
    return out


def test_batched_equals_one_by_one(ctx):
    print("batched: 6 uneven instances", flush=True)
    ins = _instances(ctx)
    probs = []
    for j, d in enumerate(ins):
        probs.append(tsk.Problem(d["tab"], d["S64"].clone(), d["S32"].clone(), d["k"], d["L"], d["T"],
                                 dtype=d["dt"], seed=300 + j))
    assert tsk.workspace_size(ctx, probs) > 0
    tsk.decompose_batched(ctx, probs)
    torch.cuda.synchronize()
    for j, (d, p) in enumerate(zip(ins, probs)):
        S64, S32 = d["S64"].clone(), d["S32"].clone()
        lam, U, tau, fl = tsk.decompose(ctx, d["tab"], S64, S32, d["k"], d["L"], d["T"], dtype=d["dt"],
                                        seed=300 + j)
        torch.cuda.synchronize()
        assert torch.equal(lam, p.lam), j
        assert torch.equal(U, p.U), j
        assert torch.equal(tau, p.tau), j
        assert torch.equal(fl, p.flags), j
        assert torch.equal(S64, p.S64), j


def test_batched_replay_and_oracle(ctx):
    print("batched: replay + oracle", flush=True)
    ins = _instances(ctx)
    S0 = [(d["S64"].clone(), d["S32"].clone()) for d in ins]
    probs = [tsk.Problem(d["tab"], d["S64"], d["S32"], d["k"], d["L"], d["T"], dtype=d["dt"], seed=9)
             for d in ins]
    tsk.decompose_batched(ctx, probs)
    first = [(p.lam.clone(), p.U.clone()) for p in probs]
    for d, (a, c) in zip(ins, S0):
        d["S64"].copy_(a)
        d["S32"].copy_(c)
    tsk.decompose_batched(ctx, probs)  # replays the recorded graph
    torch.cuda.synchronize()
    for p, (lam, U) in zip(probs, first):
        assert torch.equal(p.lam, lam) and torch.equal(p.U, U)
    # the first instance is FP64: compare with the oracle's Algorithm 1
    d = ins[0]
    n, b, B = d["inst"].n, d["tab"].b, d["tab"].B
    S_time = np.stack([oracle.sketch_factors(d["inst"].lam, d["inst"].A, d["h"][m], d["xi"][m], b)
                       for m in range(B)])
    u0 = np.stack([oracle.start_vectors_spec(9, c, d["L"], n) for c in range(d["k"])])
    r = oracle.rtpm_sketched(S_time, d["h"], d["xi"], d["k"], d["L"], d["T"], u0)
    np.testing.assert_allclose(probs[0].lam.cpu().numpy(), r.lam, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(probs[0].U.cpu().numpy(), r.U, rtol=0, atol=1e-12)


def test_batched_errors_name_the_instance(ctx):
    ins = _instances(ctx)[:2]
    bad = [tsk.Problem(d["tab"], d["S64"], d["S32"], d["k"], d["L"], d["T"], dtype=d["dt"]) for d in ins]
    bad[1].k = ins[1]["tab"].n + 1
    with pytest.raises(tsk.TskError, match="instance 1"):
        tsk.decompose_batched(ctx, bad)
