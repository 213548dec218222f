"""Hash/sign tables and start vectors (oracle side) -- test infrastructure only.

Algorithm 1 draws, for every sketch m and mode j in {1,2,3}, a hash
h_j^(m): [n] -> [b] and a Rademacher sign xi_j^(m): [n] -> {+1,-1}
(Section 2, the tensor sketch paragraph; Algorithm 1 initialisation).  The
paper asks for a 2-wise independent family; fully random tables satisfy any
k-wise requirement.  Both sides of the parity check derive them from one
counter-based generator, SplitMix64 (Steele, Lea and Flood, OOPSLA 2014),
written here from its published definition:

    z  = x + 0x9E3779B97F4A7C15
    z  = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z  = (z ^ (z >> 27)) * 0x94D049BB133111EB
    out = z ^ (z >> 31)                         (all mod 2^64)

Table entry (m, j, i):  r = mix64(mix64(seed ^ 0x68617368) + (m<<34 | j<<32 | i))
    h  = ((r >> 32) * b) >> 32       (uniform on [0, b))
    xi = -1 if bit 31 of r is set else +1

Start vector entry (comp c, restart tau, coordinate i), uniform on the sphere
(Algorithm 1 draws u_0 uniformly from the unit sphere):
    r_e = mix64(mix64(seed ^ 0x75307530) + (c<<40 | tau<<20 | (2i+e))), e in {0,1}
    U_e = (r_e >> 11) * 2^-53
    z_i = sqrt(-2 ln(1 - U_0)) * cos(2 pi U_1)        (Box-Muller)
    u   = z / ||z||_2
"""
from __future__ import annotations

import math

import numpy as np

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def mix64(x: int) -> int:
    z = (x + GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


class SplitMixStream:
    """The sequential SplitMix64 generator: state += GOLDEN, emit mix(state)."""

    def __init__(self, seed: int):
        self.state = seed & MASK

    def next(self) -> int:
        out = mix64(self.state)
        self.state = (self.state + GOLDEN) & MASK
        return out


def hash_tables(seed: int, n: int, b: int, B: int):
    """Return (h[B][3][n] uint32, xi[B][3][n] int8) per the spec above."""
    if n < 1 or B < 1 or b < 1:
        raise ValueError("n, b, B must be positive")
    base = mix64((seed ^ 0x68617368) & MASK)
    h = np.zeros((B, 3, n), dtype=np.uint32)
    xi = np.zeros((B, 3, n), dtype=np.int8)
    for m in range(B):
        for j in range(3):
            for i in range(n):
                r = mix64((base + ((m << 34) | (j << 32) | i)) & MASK)
                h[m, j, i] = ((r >> 32) * b) >> 32
                xi[m, j, i] = -1 if (r >> 31) & 1 else 1
    return h, xi


def start_vectors_spec(seed: int, comp: int, L: int, n: int) -> np.ndarray:
    """u0[L][n] for one component, per the Box-Muller spec above (FP64)."""
    base = mix64((seed ^ 0x75307530) & MASK)
    out = np.zeros((L, n), dtype=np.float64)
    for tau in range(L):
        z = []
        for i in range(n):
            key = (comp << 40) | (tau << 20) | (2 * i)
            r0 = mix64((base + key) & MASK)
            r1 = mix64((base + key + 1) & MASK)
            u0 = (r0 >> 11) * (1.0 / 9007199254740992.0)
            u1 = (r1 >> 11) * (1.0 / 9007199254740992.0)
            z.append(math.sqrt(-2.0 * math.log(1.0 - u0)) * math.cos(2.0 * math.pi * u1))
        nrm = math.sqrt(math.fsum(v * v for v in z))
        out[tau] = [v / nrm for v in z]
    return out
