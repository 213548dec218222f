"""Host check of the index algebra behind the pruned read-offs (no GPU).

The LDS transforms are Stockham passes: a pass of radix R at stride NS reads
x[j + r N/R], multiplies by W_{NS R}^{r k} (k = j mod NS), takes an R-point DFT
and writes output q to (j - k) R + k + q NS.  The pruned read-offs rely on what
the buffer holds when the last two passes are left out: group g < G = N / NS3
at positions g NS3 + k holds the NS3-point transform of the inputs congruent to
g modulo G, so that output p = sum_g W_N^{-g p} D_g[p mod NS3].  This test
emulates the passes in numpy with the kernels' radix plan (R = min(N / threads,
16) per pass, the last pass taking what is left), checks the full plan against
numpy's FFT, and then checks that identity, for every plan the read-offs use.
"""
import numpy as np
import pytest


def rmax(N, NT):
    q = N // NT
    return 16 if q >= 16 else 8 if q >= 8 else 4 if q >= 4 else 2


def plan(N, NT):
    out, ns, r = [], 1, rmax(N, NT)
    while ns < N:
        rad = r if N // ns >= r else N // ns
        out.append((ns, rad))
        ns *= rad
    return out


def stockham_pass(x, NS, R, inv):
    N = x.size
    NB = N // R
    sgn = 1.0 if inv else -1.0
    j = np.arange(NB)
    k = j % NS
    r = np.arange(R)
    v = x[j[:, None] + r[None, :] * NB] * np.exp(sgn * 2j * np.pi * np.outer(k, r) / (NS * R))
    y = v @ np.exp(sgn * 2j * np.pi * np.outer(r, r) / R)
    out = np.empty_like(x)
    out[((j - k) * R + k)[:, None] + r[None, :] * NS] = y
    return out


@pytest.mark.parametrize("N,NT", [(8192, 512), (16384, 1024), (8192, 1024), (1024, 128),
                                  (4096, 256), (256, 64), (128, 64)])
def test_groups_before_the_last_two_passes(N, NT):
    rng = np.random.default_rng(N + NT)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    passes = plan(N, NT)
    assert len(passes) >= 3
    full = x.copy()
    for ns, rad in passes:
        full = stockham_pass(full, ns, rad, inv=True)
    np.testing.assert_allclose(full, N * np.fft.ifft(x), rtol=0, atol=1e-9 * np.abs(full).max())
    part = x.copy()
    for ns, rad in passes[:-2]:
        part = stockham_pass(part, ns, rad, inv=True)
    ns3 = passes[-2][0]
    G = N // ns3
    # each group is the inverse transform of its residue class
    for g in (0, 1, G - 1):
        np.testing.assert_allclose(part[g * ns3:(g + 1) * ns3], ns3 * np.fft.ifft(x[g::G]),
                                   rtol=0, atol=1e-9 * np.abs(full).max())
    # and every output is the group sum
    p = rng.integers(0, N, 64)
    gg = np.arange(G)
    z = (np.exp(2j * np.pi * np.outer(p, gg) / N) * part[gg[None, :] * ns3 + (p % ns3)[:, None]]).sum(1)
    np.testing.assert_allclose(z, full[p], rtol=0, atol=1e-9 * np.abs(full).max())
