"""Parity of the held-out likelihood (Section 5.2, tsk_lda_heldout through the
C ABI) with the oracle's exact active-set fit.

Bars: FP64 throughout, so the mixing vectors within 1e-12 normwise relative
per document (both sides solve the same equality-constrained system on the
same support) and the log-likelihoods within 1e-12 relative.
Inputs: seeded synthetic LDA corpora (Dirichlet topics and mixtures, Poisson
lengths, some documents with one or two words), a topic matrix made positive by
mixing in a little of the uniform distribution.
"""
import numpy as np
import pytest

from oracle import heldout as H
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


def _smooth(Phi, eps):
    V = Phi.shape[0]
    return (1.0 - eps) * Phi + eps / V


@pytest.mark.parametrize("D,V,K,L,eps", [(40, 60, 5, 20.0, 1e-3), (64, 300, 10, 60.0, 1e-3),
                                         (20, 2000, 100, 150.0, 1e-4), (33, 500, 37, 8.0, 1e-2)])
def test_heldout_matches_oracle(ctx, D, V, K, L, eps):
    print(f"heldout D={D} V={V} K={K}", flush=True)
    C = lda_corpus(D=D, V=V, K=K, seed=D + K, mean_len=L, min_len=1)
    Phi = _smooth(C.Phi, eps)
    rp = torch.from_numpy(C.rowptr.astype(np.int32)).to(DEV)
    col = torch.from_numpy(C.col.astype(np.int32)).to(DEV)
    cnt = torch.from_numpy(C.cnt.astype(np.int32)).to(DEV)
    pi, ll = tsk.lda_heldout(ctx, rp, col, cnt, V, torch.from_numpy(Phi).to(DEV))
    pi, ll = pi.cpu().numpy(), ll.cpu().numpy()
    rpi, rll = H.heldout_fit(C, Phi)
    G = Phi.T @ Phi
    for d in range(D):
        assert rel(pi[d], rpi[d]) < 1e-12, (d, rel(pi[d], rpi[d]))
        assert abs(ll[d] - rll[d]) <= 1e-12 * abs(rll[d]), (d, ll[d], rll[d])
        lo, hi = C.rowptr[d], C.rowptr[d + 1]
        n = C.cnt[lo:hi].astype(np.float64)
        c = Phi[C.col[lo:hi]].T @ (n / n.sum())
        assert H.kkt_residual(G, c, pi[d]) < 1e-10


def test_heldout_at_topic_model_shape(ctx):
    """The topic-model workload's shape (V = 20000, K = 100 topics from
    Dirichlet(0.01), Poisson(150) lengths) on 300 documents, every document
    against the oracle."""
    D, V, K = 300, 20000, 100
    print(f"heldout C4 shape D={D} V={V} K={K}", flush=True)
    C = lda_corpus(D=D, V=V, K=K, seed=5, mean_len=150.0, min_len=1)
    Phi = _smooth(C.Phi, 1e-3)
    rp = torch.from_numpy(C.rowptr.astype(np.int32)).to(DEV)
    col = torch.from_numpy(C.col.astype(np.int32)).to(DEV)
    cnt = torch.from_numpy(C.cnt.astype(np.int32)).to(DEV)
    pi, ll = tsk.lda_heldout(ctx, rp, col, cnt, V, torch.from_numpy(Phi).to(DEV))
    pi, ll = pi.cpu().numpy(), ll.cpu().numpy()
    rpi, rll = H.heldout_fit(C, Phi)
    for d in range(D):
        assert rel(pi[d], rpi[d]) < 1e-12, (d, rel(pi[d], rpi[d]))
        assert abs(ll[d] - rll[d]) <= 1e-12 * abs(rll[d]), (d, ll[d], rll[d])


def test_heldout_true_topics_beat_uniform(ctx):
    """The generating topics explain held-out documents better than a topic
    matrix of uniform columns perturbed at random (average L_d)."""
    D, V, K = 200, 400, 8
    C = lda_corpus(D=D, V=V, K=K, seed=77, mean_len=80.0, min_len=1)
    rng = np.random.default_rng(3)
    rp = torch.from_numpy(C.rowptr.astype(np.int32)).to(DEV)
    col = torch.from_numpy(C.col.astype(np.int32)).to(DEV)
    cnt = torch.from_numpy(C.cnt.astype(np.int32)).to(DEV)
    _, ll_true = tsk.lda_heldout(ctx, rp, col, cnt, V, torch.from_numpy(_smooth(C.Phi, 1e-4)).to(DEV))
    R = rng.uniform(0.5, 1.5, size=(V, K))
    R /= R.sum(axis=0, keepdims=True)
    _, ll_rand = tsk.lda_heldout(ctx, rp, col, cnt, V, torch.from_numpy(R).to(DEV))
    assert float(ll_true.mean()) > float(ll_rand.mean()) + 1.0


def test_heldout_argument_errors(ctx):
    rp = torch.tensor([0, 1], dtype=torch.int32, device=DEV)
    col = torch.tensor([0], dtype=torch.int32, device=DEV)
    cnt = torch.tensor([3], dtype=torch.int32, device=DEV)
    with pytest.raises(tsk.TskError):
        tsk.lda_heldout(ctx, rp, col, cnt, 3, torch.ones((3, 4), dtype=torch.float64, device=DEV))
