"""CPU oracle for sketched tensor CP decomposition -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 reference written from the paper (Wang, Tung, Smola,
Anandkumar, "Fast and Guaranteed Tensor Decomposition via Sketching",
NIPS 2015).  It computes the definitions directly -- Eq. (1) by an explicit
scatter over all n^3 entries, Eq. (2) by circular convolution, Proposition 1
as the paper states it, Algorithm 1 step by step -- so that a reader can check
it against the paper by eye.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The library under ``paper_1506_04448_amd`` never
imports it, and it never imports the library: the two share no code.

Pinned by the ``-m "not gpu"`` tests in ``tests/test_oracle_*.py`` (identities
of Eq. (2) and Proposition 1, the injective-hash special case that reduces
every estimate to the exact dense contraction, unbiasedness by full
enumeration of hash draws, exact recovery of planted orthogonal components).
The gradients of the sketched T(u,u,u) estimate and of the sketched CP loss
(``gradients``) are pinned by central finite differences and by the
injective-hash reduction to the dense gradient.  The whitened LDA moment of
Appendix D (``lda``) is pinned by brute force over word positions, by the
closed forms of the population moments and by the explicit V^3 route.
Fast ALS (``als``, Appendix C) is pinned by the injective-hash reduction of
the two-vector estimate to the exact contraction, by its unbiasedness over
all sign (and, tiny case, hash) draws, and by exact ALS recovering an exactly
low-rank tensor.  The colliding-hash symmetric sketch (``symmetric``, Section
3.3 and Appendix B) is pinned by the equality of its full and upper-triangle
builds, exact unbiasedness of entry recovery and of both contractions over
every sign draw (which also fixes the read-off weights), and the direct
convolution route.
Parity unpinned: the full sketched power method beyond those pins (the paper
prints no worked example to compare against).
"""
from .tables import mix64, hash_tables, start_vectors_spec, SplitMixStream
from .sketch import (count_sketch, sketch_dense, circular_convolution,
                     circular_convolution_fft, sketch_rank1, sketch_rank1_fft,
                     sketch_factors)
from .contract import (median, power_update_sketch, power_update_direct,
                       tuuu_sketch, tuuu_direct, power_update, contract_uuu)
from .rtpm import rtpm_sketched, rtpm_dense, RtpmResult
from . import gradients, lda, als, symmetric
from .dense import (dense_Tuuu, dense_TIuu, residual_dense, residual_factored,
                    wrong_vectors)

__all__ = [
    "mix64", "hash_tables", "start_vectors_spec", "SplitMixStream",
    "count_sketch", "sketch_dense", "circular_convolution",
    "circular_convolution_fft", "sketch_rank1", "sketch_rank1_fft", "sketch_factors",
    "median", "power_update_sketch", "power_update_direct", "tuuu_sketch",
    "tuuu_direct", "power_update", "contract_uuu",
    "rtpm_sketched", "rtpm_dense", "RtpmResult",
    "gradients", "lda", "als", "symmetric", "dense_Tuuu", "dense_TIuu", "residual_dense", "residual_factored", "wrong_vectors",
]
