"""Sketched tensor CP decomposition on MI355X -- Python binding of libtsk.so.

Thin ctypes layer over the C ABI declared in ``include/tsk.h``: each function
has the C entry point's name without the ``tsk_`` prefix, checks the torch
tensors it is given (device, dtype, contiguity, size), passes their data
pointers and the current HIP stream, and raises :class:`TskError` on a non-OK
status.  Every step of the method runs in the library's HIP kernels; there is
no fallback: if ``libtsk.so`` is missing, importing the compute functions
raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "TskError", "lib", "library_path", "Context", "Tables", "hash_generate", "init_vectors",
    "new_sketch", "sketch_build_dense", "sketch_build_factors", "sketch_from_time",
    "sketch_export", "sketch_deflate", "power_update", "power_update_noalloc", "tune_config", "docs_route", "lda_heldout", "contract_tiuu",
    "contract_uuu",
    "decompose", "contract_tuuu_grad", "cp_loss", "Problem", "decompose_batched",
    "workspace_size", "sketch_build_docs",
    "F32", "F64",
]

F32 = 0
F64 = 1
_PKG = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_PKG, "libtsk.so")

_STATUS = {0: "TSK_OK", -1: "TSK_EINVAL", -2: "TSK_ESHAPE", -3: "TSK_ENOMEM",
           -4: "TSK_EHIP", -5: "TSK_EUNSUPPORTED"}


class TskError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} -> {_STATUS.get(status, status)}: {msg}")
        self.status = status
        self.fn = fn


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_U64 = ctypes.c_uint64
_SIGS = {
    "tsk_version": ([], ctypes.c_char_p),
    "tsk_last_error": ([], ctypes.c_char_p),
    "tsk_create": ([ctypes.POINTER(_P), _I], _I),
    "tsk_destroy": ([_P], None),
    "tsk_hash_generate": ([_U64, _I, _I, _I, _P, _P], _I),
    "tsk_init_vectors": ([_U64, _I, _I, _I, _P], _I),
    "tsk_tables_create": ([_P, _I, _I, _I, _P, _P, ctypes.POINTER(_P)], _I),
    "tsk_tables_destroy": ([_P], None),
    "tsk_sketch_build_dense": ([_P, _P, _P, _I, _P, _P, _I, _P], _I),
    "tsk_sketch_build_factors": ([_P, _P, _P, _P, _I, _P, _P, _I, _P], _I),
    "tsk_sketch_from_time": ([_P, _I, _I, _P, _P, _P, _P], _I),
    "tsk_sketch_export": ([_P, _I, _I, _P, _P, _P], _I),
    "tsk_sketch_deflate": ([_P, _P, _P, _P, _I, _P, _P, _P], _I),
    "tsk_power_update": ([_P, _P, _I, _P, _P, _I, _P, _P, _P, _P, _P], _I),
    "tsk_power_update_noalloc": ([_P, _P, _I, _P, _P, _I, _P, _P, _P, _P], _I),
    "tsk_tune_config": ([_P, _I, ctypes.c_char_p], _I),
    "tsk_docs_route": ([_P, _I], _I),
    "tsk_lda_heldout": ([_P, _P, _P, _P, _I, _I, _I, _P, _P, _P, _P], _I),
    "tsk_median_normalize": ([_P, _I, _I, _I, _I, _P, _P, _P, _P, _P], _I),
    "tsk_contract_two": ([_P, _P, _I, _P, _P, _I, _I, _P, _P, _P, _P], _I),
    "tsk_sym_tables_create": ([_P, _I, _I, _I, _P, _P, _P], _I),
    "tsk_lda_whiten": ([_P, _P, _P, _P, _I, _I, _I, ctypes.c_double, _P, _I, _P, _P, _P], _I),
    "tsk_lda_recover": ([_P, _I, _I, _I, ctypes.c_double, _P, _P, _P, _P, _P, _P], _I),
    "tsk_sym_tables_destroy": ([_P], None),
    "tsk_sym_sketch_build_dense": ([_P, _P, _P, _I, _P, _P, _P, _P, _I, _P], _I),
    "tsk_sym_contract_tiuu": ([_P, _P, _P, _P, _I, _P, _P, _P], _I),
    "tsk_sym_decompose": ([_P, _P, _P, _P, _P, _P, _I, _I, _I, _P, ctypes.c_uint64, _P, _P, _P, _P, _P], _I),
    "tsk_als": ([_P, _P, _I, _P, _P, _I, _I, _P, _P, _P, _P], _I),
    "tsk_contract_uuu": ([_P, _P, _I, _P, _P, _I, _P, _P, _P, _P], _I),
    "tsk_contract_tiuu": ([_P, _P, _I, _P, _P, _I, _P, _P, _P], _I),
    "tsk_decompose": ([_P, _P, _I, _P, _P, _I, _I, _I, _P, _U64, _P, _P, _P, _P, _I, _P], _I),
    "tsk_contract_tuuu_grad": ([_P, _P, _I, _P, _P, _I, _P, _P, _P, _P, _P, _P], _I),
    "tsk_cp_loss": ([_P, _P, _I, _P, _I, _P, _P, _P, _P, _P, _P, _P], _I),
    "tsk_decompose_batched": ([_P, _I, _P, _P], _I),
    "tsk_sketch_build_docs": ([_P, _P, _P, _P, _P, _I, _I, _P, _I, ctypes.c_double, _P, _P, _I, _P], _I),
    "tsk_workspace_size": ([_P, _I, _P, ctypes.POINTER(ctypes.c_size_t)], _I),
}


def lib() -> ctypes.CDLL:
    """Load libtsk.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise RuntimeError(f"libtsk.so not found at {library_path}: build it first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        # Load torch first so the library binds to the same HIP runtime that
        # owns torch's device memory (the two share the runtime's soname).
        import torch  # noqa: F401
        L = ctypes.CDLL(library_path)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(fn: str, status: int):
    if status != 0:
        raise TskError(fn, status, lib().tsk_last_error().decode(errors="replace"))


def _ptr(x) -> int | None:
    if x is None:
        return None
    return x.data_ptr()


def _stream(stream) -> int | None:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def _tensor(x, name, dtype, shape=None, allow_none=False):
    import torch
    if x is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not x.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(x.shape)}")
    return x


def hash_generate(seed: int, n: int, b: int, B: int):
    """Host draw of the hash/sign tables: (h uint32[B][3][n], xi int8[B][3][n])."""
    h = np.zeros((B, 3, n), dtype=np.uint32)
    xi = np.zeros((B, 3, n), dtype=np.int8)
    _check("tsk_hash_generate", lib().tsk_hash_generate(
        seed & (2 ** 64 - 1), n, b, B, h.ctypes.data, xi.ctypes.data))
    return h, xi


def init_vectors(seed: int, comp: int, L: int, n: int) -> np.ndarray:
    """Host draw of start vectors u0[L][n] (unit sphere) for one component."""
    u = np.zeros((L, n), dtype=np.float64)
    _check("tsk_init_vectors", lib().tsk_init_vectors(seed & (2 ** 64 - 1), comp, L, n,
                                                        u.ctypes.data))
    return u


class Context:
    """A library context on one HIP device."""

    def __init__(self, device: int = 0):
        h = _P()
        _check("tsk_create", lib().tsk_create(ctypes.byref(h), device))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            lib().tsk_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tables:
    """Device copy of hash/sign tables (h[B][3][n] in [0,b), xi[B][3][n] in {+-1})."""

    def __init__(self, ctx: Context, h: np.ndarray, xi: np.ndarray, b: int):
        h = np.ascontiguousarray(h, dtype=np.uint32)
        xi = np.ascontiguousarray(xi, dtype=np.int8)
        if h.ndim != 3 or h.shape[1] != 3 or xi.shape != h.shape:
            raise ValueError("tables must be [B][3][n]")
        self.B, _, self.n = h.shape
        self.b = b
        self.ctx = ctx
        t = _P()
        _check("tsk_tables_create", lib().tsk_tables_create(
            ctx.handle, self.n, b, self.B, h.ctypes.data, xi.ctypes.data, ctypes.byref(t)))
        self.handle = t

    def close(self):
        if getattr(self, "handle", None):
            lib().tsk_tables_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SymTables:
    """Device copy of colliding-hash tables (h[B][n] in [0,b), q[B][n] in
    {0,1,2,3}: sigma = i^q), Section 3.3."""

    def __init__(self, ctx: Context, h: np.ndarray, q: np.ndarray, b: int):
        h = np.ascontiguousarray(h, dtype=np.uint32)
        q = np.ascontiguousarray(q, dtype=np.uint8)
        if h.ndim != 2 or q.shape != h.shape:
            raise ValueError("symmetric tables must be [B][n]")
        self.B, self.n = h.shape
        self.b = b
        self.ctx = ctx
        t = _P()
        _check("tsk_sym_tables_create", lib().tsk_sym_tables_create(
            ctx.handle, self.n, b, self.B, h.ctypes.data, q.ctypes.data, ctypes.byref(t)))
        self.handle = t

    def close(self):
        if getattr(self, "handle", None):
            lib().tsk_sym_tables_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def new_sym_sketch(tab: SymTables, device="cuda"):
    """Allocate (s64, s32, S64, S32), each [B][b][2] (complex time domain and
    spectrum, FP64 and FP32)."""
    import torch
    shp = (tab.B, tab.b, 2)
    return (torch.zeros(shp, dtype=torch.float64, device=device), torch.zeros(shp, dtype=torch.float32, device=device),
            torch.zeros(shp, dtype=torch.float64, device=device), torch.zeros(shp, dtype=torch.float32, device=device))


def _symsk(tab, s64, s32, S64, S32):
    import torch
    shp = (tab.B, tab.b, 2)
    _tensor(s64, "s64", torch.float64, shp)
    _tensor(s32, "s32", torch.float32, shp)
    _tensor(S64, "S64", torch.float64, shp)
    _tensor(S32, "S32", torch.float32, shp)


def sym_sketch_build_dense(ctx, tab, T, s64, s32, S64, S32, accumulate=False, stream=None):
    """Eq. (5) sketches of the dense symmetric tensor T [n][n][n] (float32/64)."""
    import torch
    dt = F32 if T.dtype == torch.float32 else F64
    _tensor(T, "T", torch.float32 if dt == F32 else torch.float64, (tab.n, tab.n, tab.n))
    _symsk(tab, s64, s32, S64, S32)
    _check("tsk_sym_sketch_build_dense", lib().tsk_sym_sketch_build_dense(
        ctx.handle, tab.handle, _ptr(T), dt, _ptr(s64), _ptr(s32), _ptr(S64), _ptr(S32), int(bool(accumulate)),
        _stream(stream)))


def sym_contract_tiuu(ctx, tab, U, S32, s32, V=None, stream=None):
    """Per-sketch Re T(I,u,u) estimates V [L][B][n] (float32) on symmetric sketches."""
    import torch
    L = U.shape[0]
    _tensor(U, "U", torch.float32, (L, tab.n))
    _tensor(S32, "S32", torch.float32, (tab.B, tab.b, 2))
    _tensor(s32, "s32", torch.float32, (tab.B, tab.b, 2))
    if V is None:
        V = torch.empty((L, tab.B, tab.n), dtype=torch.float32, device=U.device)
    _tensor(V, "V", torch.float32, (L, tab.B, tab.n))
    _check("tsk_sym_contract_tiuu", lib().tsk_sym_contract_tiuu(
        ctx.handle, tab.handle, _ptr(S32), _ptr(s32), L, _ptr(U), _ptr(V), _stream(stream)))
    return V


def sym_decompose(ctx, tab, s64, s32, S64, S32, k, L, T, u0=None, seed=0, stream=None):
    """Algorithm 1 on symmetric sketches (deflated in place).
    Returns (lam [k] f64, U [k][n] f64, tau [k] i32, flags [k][L] i32)."""
    import torch
    _symsk(tab, s64, s32, S64, S32)
    _tensor(u0, "u0", torch.float64, (k, L, tab.n), allow_none=True)
    dev = S64.device
    lam = torch.empty((k,), dtype=torch.float64, device=dev)
    U = torch.empty((k, tab.n), dtype=torch.float64, device=dev)
    tau = torch.empty((k,), dtype=torch.int32, device=dev)
    flags = torch.empty((k, L), dtype=torch.int32, device=dev)
    _check("tsk_sym_decompose", lib().tsk_sym_decompose(
        ctx.handle, tab.handle, _ptr(s64), _ptr(s32), _ptr(S64), _ptr(S32), k, L, T, _ptr(u0),
        seed & (2 ** 64 - 1), _ptr(lam), _ptr(U), _ptr(tau), _ptr(flags), _stream(stream)))
    return lam, U, tau, flags


def lda_whiten(ctx, rowptr, col, cnt, D, V, K, alpha0, Omega, iters=4, stream=None):
    """Whitening of the empirical M2 (Algorithm 3) by randomized subspace
    iteration from the float64 block Omega [V][K]; returns (W [V][K], sigma [K])."""
    import torch
    for t, name in ((rowptr, "rowptr"), (col, "col"), (cnt, "cnt")):
        _tensor(t, name, torch.int32)
    _tensor(Omega, "Omega", torch.float64, (V, K))
    W = torch.empty((V, K), dtype=torch.float64, device=Omega.device)
    sig = torch.empty((K,), dtype=torch.float64, device=Omega.device)
    _check("tsk_lda_whiten", lib().tsk_lda_whiten(
        ctx.handle, _ptr(rowptr), _ptr(col), _ptr(cnt), D, V, K, float(alpha0), _ptr(Omega), iters, _ptr(W),
        _ptr(sig), _stream(stream)))
    return W, sig


def lda_recover(ctx, W, lam, U, alpha0, stream=None):
    """Algorithm 3's alpha [k] and topic vectors mu [k][V] from the CP
    decomposition (lam [k], U [k][K]) of M3(W, W, W)."""
    import torch
    V, K = W.shape
    k = lam.shape[0]
    _tensor(W, "W", torch.float64, (V, K))
    _tensor(lam, "lam", torch.float64, (k,))
    _tensor(U, "U", torch.float64, (k, K))
    alpha = torch.empty((k,), dtype=torch.float64, device=W.device)
    mu = torch.empty((k, V), dtype=torch.float64, device=W.device)
    _check("tsk_lda_recover", lib().tsk_lda_recover(
        ctx.handle, V, K, k, float(alpha0), _ptr(W), _ptr(lam), _ptr(U), _ptr(alpha), _ptr(mu), _stream(stream)))
    return alpha, mu


def lda_heldout(ctx, rowptr, col, cnt, V, Phi, stream=None):
    """Held-out likelihood (Section 5.2) of the topic matrix Phi [V][K]
    (float64) on a CSR corpus: the simplex-constrained least-squares mixing
    vectors pi [D][K] and the per-document average log-likelihoods L [D]."""
    import torch
    D = rowptr.shape[0] - 1
    K = Phi.shape[1]
    _tensor(rowptr, "rowptr", torch.int32, (D + 1,))
    _tensor(col, "col", torch.int32)
    _tensor(cnt, "cnt", torch.int32)
    _tensor(Phi, "Phi", torch.float64, (V, K))
    pi = torch.empty((D, K), dtype=torch.float64, device=Phi.device)
    ll = torch.empty((D,), dtype=torch.float64, device=Phi.device)
    _check("tsk_lda_heldout", lib().tsk_lda_heldout(
        ctx.handle, _ptr(rowptr), _ptr(col), _ptr(cnt), D, V, K, _ptr(Phi), _ptr(pi), _ptr(ll),
        _stream(stream)))
    return pi, ll


def new_sketch(tab: Tables, device="cuda"):
    """Allocate (S64 float64[B][b/2+1][2], S32 float32[B][b/2+1][2]) for `tab`."""
    import torch
    H1 = tab.b // 2 + 1
    return (torch.zeros((tab.B, H1, 2), dtype=torch.float64, device=device),
            torch.zeros((tab.B, H1, 2), dtype=torch.float32, device=device))


def _sk(tab, S64, S32, need32=False):
    import torch
    H1 = tab.b // 2 + 1
    _tensor(S64, "S64", torch.float64, (tab.B, H1, 2))
    _tensor(S32, "S32", torch.float32, (tab.B, H1, 2), allow_none=not need32)


def sketch_build_dense(ctx, tab, T, S64, S32=None, accumulate=False, stream=None):
    import torch
    if T.dtype not in (torch.float32, torch.float64):
        raise TypeError("T must be float32 or float64")
    _tensor(T, "T", T.dtype, (tab.n, tab.n, tab.n))
    _sk(tab, S64, S32)
    dt = F32 if T.dtype == torch.float32 else F64
    _check("tsk_sketch_build_dense", lib().tsk_sketch_build_dense(
        ctx.handle, tab.handle, _ptr(T), dt, _ptr(S64), _ptr(S32), int(bool(accumulate)),
        _stream(stream)))


def sketch_build_factors(ctx, tab, lam, A, S64, S32=None, accumulate=False, stream=None):
    import torch
    k = lam.shape[0]
    _tensor(lam, "lam", torch.float64, (k,))
    _tensor(A, "A", torch.float64, (k, tab.n))
    _sk(tab, S64, S32)
    _check("tsk_sketch_build_factors", lib().tsk_sketch_build_factors(
        ctx.handle, tab.handle, _ptr(lam), _ptr(A), k, _ptr(S64), _ptr(S32),
        int(bool(accumulate)), _stream(stream)))


def sketch_from_time(ctx, s_time, S64, S32=None, stream=None):
    import torch
    B, b = s_time.shape
    _tensor(s_time, "s_time", torch.float64, (B, b))
    _tensor(S64, "S64", torch.float64, (B, b // 2 + 1, 2))
    _tensor(S32, "S32", torch.float32, (B, b // 2 + 1, 2), allow_none=True)
    _check("tsk_sketch_from_time", lib().tsk_sketch_from_time(
        ctx.handle, b, B, _ptr(s_time), _ptr(S64), _ptr(S32), _stream(stream)))


def sketch_export(ctx, S64, b, s_time=None, stream=None):
    import torch
    B = S64.shape[0]
    _tensor(S64, "S64", torch.float64, (B, b // 2 + 1, 2))
    if s_time is None:
        s_time = torch.empty((B, b), dtype=torch.float64, device=S64.device)
    _tensor(s_time, "s_time", torch.float64, (B, b))
    _check("tsk_sketch_export", lib().tsk_sketch_export(
        ctx.handle, b, B, _ptr(S64), _ptr(s_time), _stream(stream)))
    return s_time


def sketch_deflate(ctx, tab, lam, U, S64, S32=None, stream=None):
    import torch
    c = lam.shape[0]
    _tensor(lam, "lam", torch.float64, (c,))
    _tensor(U, "U", torch.float64, (c, tab.n))
    _sk(tab, S64, S32)
    _check("tsk_sketch_deflate", lib().tsk_sketch_deflate(
        ctx.handle, tab.handle, _ptr(lam), _ptr(U), c, _ptr(S64), _ptr(S32), _stream(stream)))


def _spectra(tab, dt, S64, S32):
    """The FP32 path reads S32, the FP64 path reads S64; either may be absent otherwise."""
    import torch
    H1 = tab.b // 2 + 1
    _tensor(S64, "S64", torch.float64, (tab.B, H1, 2), allow_none=(dt == F32))
    _tensor(S32, "S32", torch.float32, (tab.B, H1, 2), allow_none=(dt == F64))


def _vdtype(dtype):
    import torch
    return (F32, torch.float32) if dtype in (F32, torch.float32, "f32") else (F64, torch.float64)


def power_update(ctx, tab, U_in, S64=None, S32=None, U_out=None, V=None, flags=None,
                 stream=None):
    """One power step for U_in [L][n] (float32 uses S32, float64 uses S64)."""
    import torch
    dt, tdt = _vdtype(U_in.dtype)
    L = U_in.shape[0]
    _tensor(U_in, "U_in", tdt, (L, tab.n))
    if U_out is None:
        U_out = torch.empty_like(U_in)
    _tensor(U_out, "U_out", tdt, (L, tab.n))
    _tensor(V, "V", tdt, (L, tab.B, tab.n), allow_none=True)
    _tensor(flags, "flags", torch.int32, (L,), allow_none=True)
    _spectra(tab, dt, S64, S32)
    _check("tsk_power_update", lib().tsk_power_update(
        ctx.handle, tab.handle, dt, _ptr(S64), _ptr(S32), L, _ptr(U_in), _ptr(U_out), _ptr(V),
        _ptr(flags), _stream(stream)))
    return U_out


def tune_config(ctx, mode, cache_path=None):
    """Launch-shape tuning of the context: 0 fixed rules, 1 time the candidates
    of each new shape on first use and record the fastest, 2 recorded choices
    only; ``cache_path`` names the text file the choices are read from and
    written to."""
    path = None if cache_path is None else os.fsencode(cache_path)
    _check("tsk_tune_config", lib().tsk_tune_config(ctx.handle, int(mode), path))


def docs_route(ctx, route):
    """Route of ``sketch_build_docs`` on this context: 0 a cost rule, 1 the
    per-document transforms, 2 the moment tensor on the matrix cores."""
    _check("tsk_docs_route", lib().tsk_docs_route(ctx.handle, int(route)))


def power_update_noalloc(ctx, tab, U_in, U_out, S64=None, S32=None, flags=None, stream=None):
    """The power step of ``power_update`` for callers that cannot allocate:
    the library allocates nothing (its estimates live in a static per-GPU
    array), so the caller passes the output ``U_out`` [L][n]."""
    import torch
    dt, tdt = _vdtype(U_in.dtype)
    L = U_in.shape[0]
    _tensor(U_in, "U_in", tdt, (L, tab.n))
    _tensor(U_out, "U_out", tdt, (L, tab.n))
    _tensor(flags, "flags", torch.int32, (L,), allow_none=True)
    _spectra(tab, dt, S64, S32)
    _check("tsk_power_update_noalloc", lib().tsk_power_update_noalloc(
        ctx.handle, tab.handle, dt, _ptr(S64), _ptr(S32), L, _ptr(U_in), _ptr(U_out), _ptr(flags),
        _stream(stream)))
    return U_out


def median_normalize(ctx, V, U_in, U_out=None, flags=None, stream=None):
    """Median over the B sketches of V [L][B][n] and normalisation; U_in [L][n]
    is the fallback for a zero or non-finite median vector."""
    import torch
    dt, tdt = _vdtype(V.dtype)
    L, B, n = V.shape
    _tensor(V, "V", tdt, (L, B, n))
    _tensor(U_in, "U_in", tdt, (L, n))
    if U_out is None:
        U_out = torch.empty_like(U_in)
    _tensor(U_out, "U_out", tdt, (L, n))
    _tensor(flags, "flags", torch.int32, (L,), allow_none=True)
    _check("tsk_median_normalize", lib().tsk_median_normalize(
        ctx.handle, dt, L, n, B, _ptr(V), _ptr(U_in), _ptr(U_out), _ptr(flags), _stream(stream)))
    return U_out


def contract_two(ctx, tab, X, Y, rd=0, S64=None, S32=None, V=None, stream=None):
    """Per-sketch estimates V [L][B][n] of T contracted with X[r] in mode
    (rd+1)%3 and Y[r] in mode (rd+2)%3, read off in mode rd (Proposition 1
    with two different vectors)."""
    import torch
    dt, tdt = _vdtype(X.dtype)
    L = X.shape[0]
    _tensor(X, "X", tdt, (L, tab.n))
    _tensor(Y, "Y", tdt, (L, tab.n))
    _spectra(tab, dt, S64, S32)
    if V is None:
        V = torch.empty((L, tab.B, tab.n), dtype=tdt, device=X.device)
    _tensor(V, "V", tdt, (L, tab.B, tab.n))
    _check("tsk_contract_two", lib().tsk_contract_two(
        ctx.handle, tab.handle, dt, _ptr(S64), _ptr(S32), rd, L, _ptr(X), _ptr(Y), _ptr(V),
        _stream(stream)))
    return V


def als(ctx, tab, F0, T, dtype=None, S64=None, S32=None, stream=None):
    """Fast ALS (Algorithm 2 with the update equation's pseudo-inverse) from
    the float64 initial factors F0 [3][k][n] (rows); returns (lam [k], F [3][k][n])."""
    import torch
    dtype = F32 if dtype is None else dtype
    k = F0.shape[1]
    _tensor(F0, "F0", torch.float64, (3, k, tab.n))
    _spectra(tab, dtype, S64, S32)
    F = torch.empty_like(F0)
    lam = torch.empty(k, dtype=torch.float64, device=F0.device)
    _check("tsk_als", lib().tsk_als(ctx.handle, tab.handle, dtype, _ptr(S64), _ptr(S32), k, T, _ptr(F0),
                                    _ptr(lam), _ptr(F), _stream(stream)))
    return lam, F


def contract_tiuu(ctx, tab, U, S64=None, S32=None, V=None, stream=None):
    """Per-sketch T(I,u,u) estimates V [L][B][n] (Proposition 1, no median)."""
    import torch
    dt, tdt = _vdtype(U.dtype)
    L = U.shape[0]
    _tensor(U, "U", tdt, (L, tab.n))
    _spectra(tab, dt, S64, S32)
    if V is None:
        V = torch.empty((L, tab.B, tab.n), dtype=tdt, device=U.device)
    _tensor(V, "V", tdt, (L, tab.B, tab.n))
    _check("tsk_contract_tiuu", lib().tsk_contract_tiuu(
        ctx.handle, tab.handle, dt, _ptr(S64), _ptr(S32), L, _ptr(U), _ptr(V), _stream(stream)))
    return V


def contract_uuu(ctx, tab, U, S64=None, S32=None, lam_per=None, stream=None):
    """T(u,u,u) estimates: returns (lam_med [L], lam_per [L][B]) as float64."""
    import torch
    dt, tdt = _vdtype(U.dtype)
    L = U.shape[0]
    _tensor(U, "U", tdt, (L, tab.n))
    _spectra(tab, dt, S64, S32)
    lam_med = torch.empty((L,), dtype=torch.float64, device=U.device)
    if lam_per is None:
        lam_per = torch.empty((L, tab.B), dtype=torch.float64, device=U.device)
    _tensor(lam_per, "lam_per", torch.float64, (L, tab.B))
    _check("tsk_contract_uuu", lib().tsk_contract_uuu(
        ctx.handle, tab.handle, dt, _ptr(S64), _ptr(S32), L, _ptr(U), _ptr(lam_med),
        _ptr(lam_per), _stream(stream)))
    return lam_med, lam_per


def decompose(ctx, tab, S64, S32, k, L, T, dtype=F32, u0=None, seed=0, plain=False,
              lam_out=None, U_out=None, tau_out=None, flags_out=None, stream=None):
    """Algorithm 1 for k components; S64/S32 are deflated in place.
    Returns (lam [k] f64, U [k][n] f64, tau [k] i32, flags [k][L] i32)."""
    import torch
    dt, _ = _vdtype(dtype)
    dev = S64.device
    _sk(tab, S64, S32, need32=(dt == F32))
    _tensor(u0, "u0", torch.float64, (k, L, tab.n), allow_none=True)
    if lam_out is None:
        lam_out = torch.empty((k,), dtype=torch.float64, device=dev)
    if U_out is None:
        U_out = torch.empty((k, tab.n), dtype=torch.float64, device=dev)
    if tau_out is None:
        tau_out = torch.empty((k,), dtype=torch.int32, device=dev)
    if flags_out is None:
        flags_out = torch.empty((k, L), dtype=torch.int32, device=dev)
    _tensor(lam_out, "lam_out", torch.float64, (k,))
    _tensor(U_out, "U_out", torch.float64, (k, tab.n))
    _tensor(tau_out, "tau_out", torch.int32, (k,))
    _tensor(flags_out, "flags_out", torch.int32, (k, L))
    _check("tsk_decompose", lib().tsk_decompose(
        ctx.handle, tab.handle, dt, _ptr(S64), _ptr(S32), k, L, T, _ptr(u0),
        seed & (2 ** 64 - 1), _ptr(lam_out), _ptr(U_out), _ptr(tau_out), _ptr(flags_out),
        int(bool(plain)), _stream(stream)))
    return lam_out, U_out, tau_out, flags_out


def contract_tuuu_grad(ctx, tab, U, S64=None, S32=None, scale=None, f_per=None, stream=None):
    """f(u) = med_m T(u,u,u)^(m) and its gradient for U [L][n].
    Returns (f_med [L] f64, f_per [L][B] f64, grad [L][n] in U's dtype); ``scale``
    ([L], U's dtype) multiplies each row of the gradient."""
    import torch
    dt, tdt = _vdtype(U.dtype)
    L = U.shape[0]
    _tensor(U, "U", tdt, (L, tab.n))
    _tensor(scale, "scale", tdt, (L,), allow_none=True)
    _spectra(tab, dt, S64, S32)
    f_med = torch.empty((L,), dtype=torch.float64, device=U.device)
    if f_per is None:
        f_per = torch.empty((L, tab.B), dtype=torch.float64, device=U.device)
    _tensor(f_per, "f_per", torch.float64, (L, tab.B))
    grad = torch.empty_like(U)
    _check("tsk_contract_tuuu_grad", lib().tsk_contract_tuuu_grad(
        ctx.handle, tab.handle, dt, _ptr(S64), _ptr(S32), L, _ptr(U), _ptr(scale), _ptr(f_med),
        _ptr(f_per), _ptr(grad), _stream(stream)))
    return f_med, f_per, grad


def cp_loss(ctx, tab, S64, lam, U, scale=None, grads=True, stream=None):
    """Sketched CP loss (1/B) sum_m ||s^(m)(T) - sum_i lam_i s^(m)(u_i^(x)3)||^2 and,
    with ``grads``, its gradients.  lam [k], U [k][n] (float32 or float64);
    ``scale`` (one element, same dtype) multiplies the gradients.
    Returns (loss 0-d f64, grad_lam or None, grad_U or None)."""
    import torch
    dt, tdt = _vdtype(U.dtype)
    k = U.shape[0]
    _tensor(S64, "S64", torch.float64, (tab.B, tab.b // 2 + 1, 2))
    _tensor(lam, "lam", tdt, (k,))
    _tensor(U, "U", tdt, (k, tab.n))
    _tensor(scale, "scale", tdt, (1,), allow_none=True)
    loss = torch.empty((), dtype=torch.float64, device=U.device)
    g_lam = torch.empty_like(lam) if grads else None
    g_U = torch.empty_like(U) if grads else None
    _check("tsk_cp_loss", lib().tsk_cp_loss(
        ctx.handle, tab.handle, dt, _ptr(S64), k, _ptr(lam), _ptr(U), _ptr(scale), _ptr(loss),
        _ptr(g_lam), _ptr(g_U), _stream(stream)))
    return loss, g_lam, g_U


class _CProblem(ctypes.Structure):
    _fields_ = [("tab", _P), ("dtype", _I), ("S64", _P), ("S32", _P), ("k", _I), ("L", _I),
                ("T", _I), ("u0", _P), ("seed", _U64), ("lam_out", _P), ("U_out", _P),
                ("tau_out", _P), ("flags_out", _P)]


class Problem:
    """One instance of a batched decomposition (tsk_problem): its tables and
    sketches, k, L, T, the precision of the power steps, optional start
    vectors, and the outputs (allocated here when not given)."""

    def __init__(self, tab, S64, S32, k, L, T, dtype=F32, u0=None, seed=0, lam_out=None,
                 U_out=None, tau_out=None, flags_out=None):
        import torch
        dt, _ = _vdtype(dtype)
        dev = S64.device
        _sk(tab, S64, S32, need32=(dt == F32))
        _tensor(u0, "u0", torch.float64, (k, L, tab.n), allow_none=True)
        self.tab, self.S64, self.S32, self.k, self.L, self.T = tab, S64, S32, k, L, T
        self.dtype, self.u0, self.seed = dt, u0, seed
        self.lam = lam_out if lam_out is not None else torch.empty((k,), dtype=torch.float64, device=dev)
        self.U = U_out if U_out is not None else torch.empty((k, tab.n), dtype=torch.float64, device=dev)
        self.tau = tau_out if tau_out is not None else torch.empty((k,), dtype=torch.int32, device=dev)
        self.flags = flags_out if flags_out is not None else torch.empty((k, L), dtype=torch.int32,
                                                                         device=dev)
        _tensor(self.lam, "lam_out", torch.float64, (k,))
        _tensor(self.U, "U_out", torch.float64, (k, tab.n))
        _tensor(self.tau, "tau_out", torch.int32, (k,))
        _tensor(self.flags, "flags_out", torch.int32, (k, L))

    def _c(self):
        return _CProblem(self.tab.handle, self.dtype, _ptr(self.S64), _ptr(self.S32), self.k, self.L,
                         self.T, _ptr(self.u0), self.seed & (2 ** 64 - 1), _ptr(self.lam),
                         _ptr(self.U), _ptr(self.tau), _ptr(self.flags))


def _problems(problems):
    arr = (_CProblem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = p._c()
    return arr


def decompose_batched(ctx, problems, stream=None):
    """Algorithm 1 for every Problem in ``problems`` in one graph launch; each
    problem's sketches are deflated in place and its outputs filled."""
    arr = _problems(problems)
    _check("tsk_decompose_batched", lib().tsk_decompose_batched(
        ctx.handle, len(problems), ctypes.cast(arr, _P), _stream(stream)))
    return problems


def workspace_size(ctx, problems) -> int:
    """Device workspace bytes tsk_decompose_batched keeps for ``problems``."""
    arr = _problems(problems)
    out = ctypes.c_size_t(0)
    _check("tsk_workspace_size", lib().tsk_workspace_size(
        ctx.handle, len(problems), ctypes.cast(arr, _P), ctypes.byref(out)))
    return int(out.value)


def sketch_build_docs(ctx, tab, rowptr, col, cnt, V, W, alpha0, S64, S32=None, accumulate=False,
                      stream=None):
    """Sketches of the whitened LDA moment M3(W,W,W) from CSR word counts
    (rowptr int32 [D+1], col/cnt int32 [nnz]) and W [V][K] (float32 or float64)."""
    import torch
    D = rowptr.shape[0] - 1
    _tensor(rowptr, "rowptr", torch.int32, (D + 1,))
    _tensor(col, "col", torch.int32)
    _tensor(cnt, "cnt", torch.int32, tuple(col.shape))
    dt, tdt = _vdtype(W.dtype)
    _tensor(W, "W", tdt, (V, tab.n))
    _sk(tab, S64, S32)
    _check("tsk_sketch_build_docs", lib().tsk_sketch_build_docs(
        ctx.handle, tab.handle, _ptr(rowptr), _ptr(col), _ptr(cnt), D, V, _ptr(W), dt, float(alpha0),
        _ptr(S64), _ptr(S32), int(bool(accumulate)), _stream(stream)))
