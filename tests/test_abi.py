"""C ABI checks that need no GPU: the library loads, exports every symbol
the header declares, and rejects bad arguments on the host before any
device work."""
import ctypes as C
import os
import re

import pytest

from paper_2603_21444_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "spgemm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(spgemm_\w+)\s*\(", txt, re.M)))


def test_every_declared_symbol_is_exported():
    L = binding.lib()
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert sorted(binding.EXPORTS) == names


def test_status_strings():
    assert binding.status_string(0) == "ok"
    for code in range(1, 9):
        assert binding.status_string(code) not in ("ok", "unknown status")
    assert binding.status_string(99) == "unknown status"


def test_workspace_size_is_host_only_and_monotone():
    s1 = binding.workspace_size(1000, 1000, 1000)
    s2 = binding.workspace_size(2000, 1000, 1000)
    s3 = binding.workspace_size(0, 0, 0)
    assert 0 < s3 < s1 < s2
    b = C.c_size_t()
    assert binding.lib().spgemm_workspace_size(-1, 5, 5, C.byref(b)) == binding.SPG_ERR_ARG


def test_tuning_roundtrip_and_rejection():
    L = binding.lib()
    p = C.c_void_p()
    assert L.spgemm_plan_create(0, C.byref(p)) == 0
    t = binding.default_tuning()
    assert L.spgemm_plan_set_tuning(p, C.byref(t)) == 0
    t.lanes[3] = 3
    assert L.spgemm_plan_set_tuning(p, C.byref(t)) == binding.SPG_ERR_ARG
    t = binding.default_tuning()
    t.max_window = 0
    assert L.spgemm_plan_set_tuning(p, C.byref(t)) == binding.SPG_ERR_ARG
    L.spgemm_plan_destroy(p)
    assert L.spgemm_plan_create(0, None) == binding.SPG_ERR_ARG


def _csr(m, n, nnz):
    # host-side descriptors only: shape checks fail before any pointer is used
    return binding.SpgCsr(m, n, nnz, 16, 16, 16)


@pytest.mark.parametrize("K", [0, 17])
def test_symbolic_rejects_bad_part_count(K):
    L = binding.lib()
    p = C.c_void_p()
    L.spgemm_plan_create(0, C.byref(p))
    A = (binding.SpgCsr * 1)(_csr(4, 5, 1))
    B = (binding.SpgCsr * 1)(_csr(5, 6, 1))
    nnz = C.c_int64()
    rc = L.spgemm_symbolic(p, K, A, B, C.c_void_p(16), C.byref(nnz), -1, C.c_void_p(16), 1 << 20, None)
    assert rc == binding.SPG_ERR_ARG
    L.spgemm_plan_destroy(p)


def test_symbolic_rejects_shape_mismatch():
    L = binding.lib()
    p = C.c_void_p()
    L.spgemm_plan_create(0, C.byref(p))
    A = (binding.SpgCsr * 1)(_csr(4, 5, 1))
    B = (binding.SpgCsr * 1)(_csr(6, 6, 1))
    nnz = C.c_int64()
    rc = L.spgemm_symbolic(p, 1, A, B, C.c_void_p(16), C.byref(nnz), -1, C.c_void_p(16), 1 << 20, None)
    assert rc == binding.SPG_ERR_SHAPE
    # batched parts must share m and n
    A2 = (binding.SpgCsr * 2)(_csr(4, 5, 1), _csr(3, 5, 1))
    B2 = (binding.SpgCsr * 2)(_csr(5, 6, 1), _csr(5, 6, 1))
    rc = L.spgemm_symbolic(p, 2, A2, B2, C.c_void_p(16), C.byref(nnz), -1, C.c_void_p(16), 1 << 20, None)
    assert rc == binding.SPG_ERR_SHAPE
    # merge operands must share the shape
    P = (binding.SpgCsr * 2)(_csr(4, 5, 1), _csr(4, 6, 1))
    rc = L.spgemm_merge(p, 2, P, 0, C.c_void_p(16), C.byref(nnz), -1, None, None, C.c_void_p(16), 1 << 20, None)
    assert rc == binding.SPG_ERR_SHAPE
    L.spgemm_plan_destroy(p)


def test_symbolic_rejects_small_workspace():
    L = binding.lib()
    p = C.c_void_p()
    L.spgemm_plan_create(0, C.byref(p))
    A = (binding.SpgCsr * 1)(_csr(4, 5, 1))
    B = (binding.SpgCsr * 1)(_csr(5, 6, 1))
    nnz = C.c_int64()
    rc = L.spgemm_symbolic(p, 1, A, B, C.c_void_p(16), C.byref(nnz), -1, C.c_void_p(16), 64, None)
    assert rc == binding.SPG_ERR_WORKSPACE
    rc = L.spgemm_symbolic(p, 1, A, B, C.c_void_p(16), C.byref(nnz), -1, None, 1 << 30, None)
    assert rc == binding.SPG_ERR_WORKSPACE
    L.spgemm_plan_destroy(p)


def test_numeric_before_symbolic_is_rejected():
    L = binding.lib()
    p = C.c_void_p()
    L.spgemm_plan_create(0, C.byref(p))
    A = (binding.SpgCsr * 1)(_csr(4, 5, 1))
    B = (binding.SpgCsr * 1)(_csr(5, 6, 1))
    rc = L.spgemm_numeric(p, 1, A, B, 0, C.c_void_p(16), C.c_void_p(16), None)
    assert rc == binding.SPG_ERR_ARG
    L.spgemm_plan_destroy(p)
