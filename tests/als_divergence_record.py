"""Record: is the divergence of fast ALS (Algorithm 2, Appendix C) on the
paper's full-rank tensors at b = 2^16 the method or the kernels?

One cell of the accuracy table (n = 1000 full rank, sigma = 0.1, B = 40,
b = 65536, k = 10, the benchmark's tables and start factors).  The GPU builds
the sketches, exports them in FP64 and runs its FP32 ALS for T = 1 .. 30
sweeps; the oracle then runs its FP64 ALS from the same start factors on the
same exported sketches.  Both lambda sequences are printed sweep by sweep.

  python tests/als_divergence_record.py gpu /tmp/als_cell.npz     (on the GPU)
  python tests/als_divergence_record.py oracle /tmp/als_cell.npz  (CPU, the file the first run wrote)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

N, K, SIGMA, BCNT, LOGB, SWEEPS = 1000, 10, 0.1, 40, 16, 30


def gpu(out):
    import torch
    import paper_1506_04448_amd as tsk
    from paper_1506_04448_amd.workloads import full_rank_tensor
    dev = torch.device("cuda:0")
    b = 1 << LOGB
    X = full_rank_tensor(N, SIGMA, seed=5, device=dev)
    ctx = tsk.Context(0)
    h, xi = tsk.hash_generate(100 + BCNT + LOGB, N, b, BCNT)
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, dev)
    tsk.sketch_build_dense(ctx, tab, X.T, S64, S32)
    S_time = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    F0 = np.random.default_rng(11).standard_normal((3, K, N))
    lam = []
    for t in range(1, SWEEPS + 1):
        l, _ = tsk.als(ctx, tab, torch.from_numpy(F0).to(dev), t, dtype=tsk.F32, S32=S32)
        lam.append(l.cpu().numpy())
        print(f"gpu sweep {t}: max lambda {np.abs(lam[-1]).max():.4g}", flush=True)
    np.savez_compressed(out, S_time=S_time, h=h, xi=xi, F0=F0, lam_gpu=np.array(lam), V_true=X.V[:K])
    tab.close()
    ctx.close()


def oracle_side(path):
    from oracle import als
    from oracle.contract import median
    d = np.load(path)
    S, h, xi, F0, lam_gpu = d["S_time"], d["h"], d["xi"], d["F0"], d["lam_gpu"]
    F = np.array(F0, dtype=np.float64, copy=True)
    print("# Fast ALS on the same FP64 sketches (n=1000 full rank, sigma=0.1, B=40, b=65536, k=10)")
    print("# sweep | oracle FP64: max |lambda|, min |lambda| | GPU FP32: max |lambda|, min |lambda| | "
          "max relative difference of the lambdas")
    for t in range(SWEEPS):
        for rd in range(3):
            Xf, Yf = F[(rd + 1) % 3], F[(rd + 2) % 3]
            V = np.stack([als.contract_two(S[m], h[m], xi[m], Xf, Yf, rd) for m in range(S.shape[0])], axis=1)
            lam, F[rd] = als.als_update(median(V, axis=1), Xf, Yf)
        g = lam_gpu[t]
        diff = np.max(np.abs(np.sort(np.abs(lam)) - np.sort(np.abs(g))) / np.maximum(np.sort(np.abs(lam)), 1e-300))
        print(f"{t + 1} | {np.abs(lam).max():.6g}, {np.abs(lam).min():.6g} | {np.abs(g).max():.6g}, "
              f"{np.abs(g).min():.6g} | {diff:.3g}", flush=True)


if __name__ == "__main__":
    if sys.argv[1] == "gpu":
        gpu(sys.argv[2])
    else:
        oracle_side(sys.argv[2])
