"""The launch-shape tuner (tsk_tune_config), through the C ABI.

A tuned run (mode 1) times the candidate shapes and records its choices in a
cache file; a later context reading that file (mode 2) must reproduce the
tuned results bit for bit.  Whatever build shape is chosen, the sketch must
still equal Eq. (1) at the FP64 bar, and the restart grouping of a
decomposition must not change any bit of its result.
"""
import numpy as np
import pytest

import oracle
from paper_1506_04448_amd.workloads import planted_tensor

torch = pytest.importorskip("torch")
import paper_1506_04448_amd as tsk  # noqa: E402
from parity_rules import rel  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N, BLEN, BCNT, K, L, T = 60, 4096, 6, 3, 8, 6


def _run(mode, path, P, h, xi, S_given=None):
    ctx = tsk.Context(0)
    tsk.tune_config(ctx, mode, None if path is None else str(path))
    tab = tsk.Tables(ctx, h, xi, BLEN)
    S64, S32 = tsk.new_sketch(tab, DEV)
    if S_given is None:
        tsk.sketch_build_dense(ctx, tab, torch.from_numpy(P.T).to(DEV), S64, S32)
    else:
        S64.copy_(S_given[0])
        S32.copy_(S_given[1])
    S0 = (S64.clone(), S32.clone())
    lam, U, _, _ = tsk.decompose(ctx, tab, S64, S32, K, L, T, dtype=tsk.F32, seed=3)
    torch.cuda.synchronize()
    out = (S0, lam.clone(), U.clone(), tsk.sketch_export(ctx, S0[0], BLEN).cpu().numpy())
    tab.close()
    ctx.close()
    return out


def _cache(path):
    return dict((ln.split()[0], [int(x) for x in ln.split()[1:]])
                for ln in path.read_text().splitlines() if ln.strip())


def test_tuned_choices_are_cached_and_reproduced(tmp_path):
    print("tune: fresh, cached, forced", flush=True)
    path = tmp_path / "tune.txt"
    P = planted_tensor(N, K, noise=0.05, seed=9)
    h, xi = tsk.hash_generate(9, N, BLEN, BCNT)
    ref = np.stack([oracle.sketch_dense(P.T, h[m], xi[m], BLEN) for m in range(BCNT)])

    fresh = _run(1, path, P, h, xi)
    table = _cache(path)
    kinds = sorted(k.split(":")[0] for k in table)
    assert kinds == ["build", "decompose"], table
    assert rel(fresh[3], ref) < 1e-12

    cached = _run(2, path, P, h, xi)
    assert torch.equal(fresh[0][0], cached[0][0]) and torch.equal(fresh[0][1], cached[0][1])
    assert torch.equal(fresh[1], cached[1]) and torch.equal(fresh[2], cached[2])

    # another recorded choice: one sketch per work-group, 8 slabs, 3 restart groups
    forced = {k: ([1, 8] if k.startswith("build:") else [3]) for k in table}
    path.write_text("".join(f"{k} {' '.join(map(str, v))}\n" for k, v in forced.items())
                    + "not-a-key-line\n")
    other = _run(2, path, P, h, xi)
    assert rel(other[3], ref) < 1e-12
    # restart groups change no bit: the rule's grouping on the same sketch
    rules = _run(0, None, P, h, xi, S_given=other[0])
    assert torch.equal(rules[1], other[1]) and torch.equal(rules[2], other[2])


def test_tuned_build_of_integer_tensor_is_exact(tmp_path):
    """Bucket sums of small integers are exact in the fixed-point build, so
    every build shape the tuner may pick gives Eq. (1) to the FP64 round trip."""
    path = tmp_path / "tune_int.txt"
    rng = np.random.default_rng(21)
    n, b, B = 40, 1024, 4
    Ti = rng.integers(-8, 9, size=(n, n, n)).astype(np.float64)
    h, xi = tsk.hash_generate(21, n, b, B)
    ctx = tsk.Context(0)
    tsk.tune_config(ctx, 1, str(path))
    tab = tsk.Tables(ctx, h, xi, b)
    S64, S32 = tsk.new_sketch(tab, DEV)
    tsk.sketch_build_dense(ctx, tab, torch.from_numpy(Ti).to(DEV), S64, S32)
    got = tsk.sketch_export(ctx, S64, b).cpu().numpy()
    ref = np.stack([oracle.sketch_dense(Ti, h[m], xi[m], b) for m in range(B)])
    assert np.abs(got - ref).max() < 1e-9
    assert any(k.startswith("build:") for k in _cache(path))
    tab.close()
    ctx.close()


def test_tune_config_rejects_bad_mode():
    ctx = tsk.Context(0)
    with pytest.raises(tsk.TskError):
        tsk.tune_config(ctx, 3)
    ctx.close()
