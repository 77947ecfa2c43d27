"""The C ABI: libltn loads without a GPU and exports every function that
include/ltn.h declares (no device call is made here)."""
import ctypes
import os
import re

from paper_2205_00393_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "ltn.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ltn_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_the_header():
    assert set(declared()) == set(_lib.SIGNATURES)


def test_error_reporting_without_gpu():
    L = _lib.lib()
    assert L.ltn_version().decode().startswith("ltn")
    st = L.ltn_plan_describe(None, None)
    assert st == -1 and "NULL" in L.ltn_last_error().decode()
    # device entry points refuse an unbound or NULL plan before touching HIP
    assert L.ltn_execute_range(None, 0, 1, 0, None) == -5


def test_permute_argument_checks_without_gpu():
    """ltn_permute rejects bad arguments on the host, before any HIP call:
    a non-permutation, in == out, and buffers that are not 16-byte aligned
    (the kernel moves 16-byte pairs). The pointers are never dereferenced."""
    import ctypes as C
    L = _lib.lib()
    perm = (C.c_int32 * 3)(2, 0, 1)
    bad = (C.c_int32 * 3)(0, 0, 1)
    assert L.ltn_permute(C.c_void_p(4096), C.c_void_p(8192), 3, bad, 1, None) == -1
    assert "permutation" in L.ltn_last_error().decode()
    assert L.ltn_permute(C.c_void_p(4096), C.c_void_p(4096), 3, perm, 1, None) == -1
    assert L.ltn_permute(C.c_void_p(4104), C.c_void_p(8192), 3, perm, 1, None) == -1
    assert "aligned" in L.ltn_last_error().decode()
    assert L.ltn_permute(C.c_void_p(4096), C.c_void_p(8200), 3, perm, 1, None) == -1
    assert "aligned" in L.ltn_last_error().decode()


def test_kernel_names_without_gpu():
    """Kernel choices are named on the host: the complex64 tiles 10-15 and
    split-K tiles 4, 5 and 7 are the three-product form (c64_3m_*, splitk_3m_*),
    tiles 0-9 and split-K 0-3 and 6 the direct form; a split kind has no name in
    complex64 mode and choices past the tables are "?"."""
    import paper_2205_00393_amd as P
    direct = [P.kernel_name(1, c) for c in range(10)]
    three = [P.kernel_name(1, c) for c in range(10, 16)]
    assert all(n.startswith("c64_") and "_3m_" not in n for n in direct)
    assert all(n.startswith("c64_3m_") for n in three)
    assert len(set(direct + three)) == 16
    assert P.kernel_name(1, 16) == "?" and P.kernel_name(1, -1) == "?"
    assert [P.kernel_name(5, c) for c in range(8)][3:] == \
        ["splitk_128x64x16", "splitk_3m_128x64x16", "splitk_3m_128x32x16", "splitk_64x32x16",
         "splitk_3m_64x64x16"]
    assert P.kernel_name(5, 8) == "?"
    assert P.kernel_name(2, 0, "c64") == "?"
    assert P.kernel_name(2, 16, "split_bf16") == "split_dma1x4_128x128x16"
    assert P.kernel_name(3, 1) == "narrow_rows" and P.kernel_name(4, 0) == "split_sum"
    assert P.kernel_name(0, -1) == "generic" and P.kernel_name(9, 0) == "?"
