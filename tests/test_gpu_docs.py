"""Parity of the document build (sketches of the whitened LDA moment
M3(W,W,W) from CSR word counts, HIP path through the C ABI) with the oracle,
which forms the K^3 tensor from the per-document terms and sketches it by
Eq. (1).  Both routes of the library run every case: route 1 sketches each
rank-1 term through transforms (Section 3.2), route 2 forms the moment
tensor on the matrix cores and sketches it by Eq. (1).

Bars: FP64 W within 1e-12 normwise relative per sketch; FP32 W within 1e-5.
Inputs: seeded synthetic LDA corpora (Dirichlet topics and mixtures,
Poisson lengths; some documents shorter than three words), random W.
"""
import numpy as np
import pytest

from oracle import lda as olda
from paper_1506_04448_amd.workloads import lda_corpus

torch = pytest.importorskip("torch")
import paper_1506_04448_amd as tsk  # noqa: E402
from parity_rules import rel  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    c = tsk.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _dev(C):
    return (torch.from_numpy(C.rowptr.astype(np.int32)).to(DEV),
            torch.from_numpy(C.col.astype(np.int32)).to(DEV),
            torch.from_numpy(C.cnt.astype(np.int32)).to(DEV))


@pytest.mark.parametrize("D,V,K,L,b,B,dt", [(300, 40, 5, 8.0, 1024, 4, np.float64),
                                            (200, 60, 7, 12.0, 256, 3, np.float64),
                                            (400, 200, 20, 30.0, 16384, 3, np.float32),
                                            (30, 300, 100, 12.0, 4096, 2, np.float32),
                                            (150, 80, 9, 6.0, 8192, 2, np.float64),
                                            # the LDA workload's sketch shape: K = 100, b = 16384, B = 8
                                            (12, 300, 100, 40.0, 16384, 8, np.float32),
                                            (12, 300, 100, 40.0, 16384, 8, np.float64),
                                            # the largest K the build takes (two column groups of the
                                            # moment route's word product, 129 columns for its documents)
                                            (6, 130, 128, 12.0, 1024, 2, np.float32),
                                            (6, 130, 128, 12.0, 1024, 2, np.float64)])
@pytest.mark.parametrize("route", [1, 2])
def test_docs_build_matches_oracle(ctx, D, V, K, L, b, B, dt, route):
    print(f"docs D={D} V={V} K={K} b={b} B={B} {np.dtype(dt).name} route {route}", flush=True)
    tsk.docs_route(ctx, route)
    C = lda_corpus(D=D, V=V, K=K, seed=D + V, mean_len=L, min_len=1)
    alpha0 = float(C.alpha.sum())
    rng = np.random.default_rng(K)
    W = (rng.standard_normal((V, K)) / np.sqrt(V)).astype(dt)
    h, xi = tsk.hash_generate(7 + K, K, b, B)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    rp, col, cnt = _dev(C)
    tsk.sketch_build_docs(ctx, tab, rp, col, cnt, V, torch.from_numpy(W).to(DEV), alpha0, S64, S32)
    got = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    ref = olda.sketch_docs(C, W.astype(np.float64), alpha0, h, xi, b)
    tol = 1e-12 if dt == np.float64 else 1e-5
    for m in range(B):
        assert rel(got[m], ref[m]) < tol, (m, rel(got[m], ref[m]))
    np.testing.assert_array_equal(S32.cpu().numpy(), S64.cpu().numpy().astype(np.float32))
    # accumulate adds the same sketch again
    tsk.sketch_build_docs(ctx, tab, rp, col, cnt, V, torch.from_numpy(W).to(DEV), alpha0, S64, S32,
                          accumulate=True)
    got2 = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    assert rel(got2, 2 * ref) < tol
    tsk.docs_route(ctx, 0)


@pytest.mark.parametrize("route", [1, 2])
def test_docs_build_all_short_documents_give_zero(ctx, route):
    tsk.docs_route(ctx, route)
    C = lda_corpus(D=20, V=10, K=3, seed=1, mean_len=0.5, min_len=1)
    lens = np.array([C.cnt[C.rowptr[d]:C.rowptr[d + 1]].sum() for d in range(20)])
    keep = lens < 3
    # keep only documents shorter than three words
    rows = [np.arange(C.rowptr[d], C.rowptr[d + 1]) for d in range(20) if keep[d]]
    rowptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    idx = np.concatenate(rows) if rows else np.zeros(0, dtype=np.int64)
    h, xi = tsk.hash_generate(3, 3, 256, 2)
    tab = tsk.Tables(ctx, h, xi, 256)
    S64, S32 = tsk.new_sketch(tab, DEV)
    S64.fill_(7.0)
    W = torch.randn((10, 3), dtype=torch.float64, device=DEV)
    tsk.sketch_build_docs(ctx, tab, torch.from_numpy(rowptr).to(DEV),
                          torch.from_numpy(C.col[idx].astype(np.int32)).to(DEV),
                          torch.from_numpy(C.cnt[idx].astype(np.int32)).to(DEV), 10, W, 1.0, S64, S32)
    tsk.docs_route(ctx, 0)
    assert float(S64.abs().max()) == 0.0


def test_docs_build_argument_errors(ctx):
    h, xi = tsk.hash_generate(3, 4, 256, 2)
    tab = tsk.Tables(ctx, h, xi, 256)
    S64, S32 = tsk.new_sketch(tab, DEV)
    rp = torch.tensor([0, 1], dtype=torch.int32, device=DEV)
    col = torch.tensor([0], dtype=torch.int32, device=DEV)
    cnt = torch.tensor([3], dtype=torch.int32, device=DEV)
    W = torch.zeros((5, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(tsk.TskError, match="alpha0"):
        tsk.sketch_build_docs(ctx, tab, rp, col, cnt, 5, W, -1.0, S64, S32)
    with pytest.raises(ValueError):
        tsk.sketch_build_docs(ctx, tab, rp, col, cnt, 5, W[:, :3].contiguous(), 1.0, S64, S32)
    with pytest.raises(tsk.TskError, match="route"):
        tsk.docs_route(ctx, 3)
