"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, its host-only randomness matches the oracle bit for bit, and
argument errors come back as status codes before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1506_04448_amd as tsk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsk.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tsk_[a-z0-9_]+)\s*\(", src)))


def test_library_loads_and_exports_every_declared_symbol():
    L = tsk.lib()
    names = _declared_functions()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding knows the signature of each
    assert set(names) <= set(tsk._SIGS), set(names) - set(tsk._SIGS)
    assert L.tsk_version().startswith(b"tsk")


@pytest.mark.parametrize("seed,n,b,B", [(0, 50, 1024, 4), (1, 200, 16384, 10), (7, 1, 64, 1),
                                        (2**64 - 1, 33, 4096, 64), (3, 17, 1000, 3)])
def test_hash_tables_bit_exact_with_oracle(seed, n, b, B):
    h, xi = tsk.hash_generate(seed, n, b, B)
    ho, xo = oracle.hash_tables(seed, n, b, B)
    np.testing.assert_array_equal(h, ho)
    np.testing.assert_array_equal(xi, xo)


@pytest.mark.parametrize("seed,comp,L,n", [(0, 0, 10, 50), (9, 3, 5, 200), (2**63, 1, 2, 1)])
def test_start_vectors_match_oracle(seed, comp, L, n):
    u = tsk.init_vectors(seed, comp, L, n)
    uo = oracle.start_vectors_spec(seed, comp, L, n)
    # same libm on the same host: equal to the last bit or within 2 ulp
    np.testing.assert_allclose(u, uo, rtol=0, atol=4e-16)


def test_host_argument_errors_return_status():
    L = tsk.lib()
    h = np.zeros((1, 3, 4), dtype=np.uint32)
    xi = np.zeros((1, 3, 4), dtype=np.int8)
    assert L.tsk_hash_generate(0, 0, 64, 1, h.ctypes.data, xi.ctypes.data) == -1
    assert L.tsk_hash_generate(0, 4, 64, 1, None, xi.ctypes.data) == -1
    assert b"null" in L.tsk_last_error()
    u = np.zeros(8)
    assert L.tsk_init_vectors(0, 0, 0, 8, u.ctypes.data) == -1
    # compute entry points reject a null context before touching any device
    assert L.tsk_power_update(None, None, 0, None, None, 1, None, None, None, None, None) == -1
    assert L.tsk_power_update_noalloc(None, None, 0, None, None, 1, None, None, None, None) == -1
    assert L.tsk_tune_config(None, 1, None) == -1
    assert L.tsk_docs_route(None, 1) == -1
    assert L.tsk_decompose(None, None, 0, None, None, 1, 1, 1, None, 0, None, None, None, None,
                           0, None) == -1
    assert L.tsk_sketch_build_dense(None, None, None, 0, None, None, 0, None) == -1
    assert L.tsk_sketch_export(None, 64, 1, None, None, None) == -1
    out = ctypes.c_void_p()
    assert L.tsk_tables_create(None, 4, 64, 1, h.ctypes.data, xi.ctypes.data,
                               ctypes.byref(out)) == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(tsk, "_lib", None)
    monkeypatch.setattr(tsk, "library_path", str(tmp_path / "libtsk.so"))
    with pytest.raises(RuntimeError, match="not found"):
        tsk.lib()


def test_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1506_04448_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "oracle/" not in txt, f
