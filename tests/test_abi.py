"""C-ABI checks that need no GPU: the library loads, exports every function
include/figaro.h declares, and rejects malformed join trees before touching
device memory."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2204_00525_amd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = "".join(open(os.path.join(ROOT, "include", h)).read()
                  for h in sorted(os.listdir(os.path.join(ROOT, "include"))) if h.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(figaro_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = F.lib()
    names = _declared()
    assert "figaro_r" in names and "figaro_plan_create" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []


def _descs(spec):
    """spec: list of (attrs, ncols, parent); keys point at a dummy address that
    must never be read because validation fails first."""
    keep = []
    arr = (F.RelationDesc * len(spec))()
    for i, (attrs, ncols, parent) in enumerate(spec):
        a = np.asarray(attrs, dtype=np.int32)
        keep.append(a)
        arr[i].rows = 5
        arr[i].num_keys = len(attrs)
        arr[i].key_attr = a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        arr[i].key_cols = ctypes.c_void_p(0x1000)
        arr[i].key_dtype = 4
        arr[i].num_cols = ncols
        arr[i].parent = parent
    return arr, keep


@pytest.mark.parametrize("spec,status", [
    ([([0], 2, -1), ([0], 2, -1)], "ENOTTREE"),                     # two roots
    ([([0], 2, 1), ([0], 2, 0)], "ENOTTREE"),                       # cycle, no root
    ([([0], 2, -1), ([0], 2, 5)], "ENOTTREE"),                      # parent out of range
    ([([0], 2, -1), ([0, 1], 2, 0), ([1], 2, 1), ([0], 2, 2)], "ENOTTREE"),  # attr 0 not connected
    ([([0, 9], 2, -1), ([0], 2, 0)], "EUNSHARED_KEY"),              # key 9 shared with nobody
    ([([0], 0, -1), ([0], 2, 0)], "EINVAL"),                        # no data columns
    ([([0, 0], 2, -1), ([0], 2, 0)], "EINVAL"),                     # repeated attribute
])
def test_plan_rejects_malformed_trees(spec, status):
    L = F.lib()
    arr, keep = _descs(spec)
    h = ctypes.c_void_p()
    opts = F.PlanOptions(0, 0, 1, 0, 1)
    st = L.figaro_plan_create(ctypes.byref(h), len(spec), arr, ctypes.byref(opts), None)
    assert F.STATUS_NAMES[st] == status
    assert not h.value
    assert L.figaro_last_error(None)


def test_plan_rejects_null_arguments():
    L = F.lib()
    h = ctypes.c_void_p()
    assert F.STATUS_NAMES[L.figaro_plan_create(ctypes.byref(h), 0, None, None, None)] == "EINVAL"
    assert L.figaro_plan_num_cols(None) == -1
    assert F.STATUS_NAMES[L.figaro_r(None, None, None, None, None)] == "EINVAL"


def test_batch_rejects_bad_plans():
    """figaro_batch_create validates its plans before touching the GPU."""
    import ctypes
    import paper_2204_00525_amd as F
    import synth
    L = F.lib()
    h = ctypes.c_void_p()
    assert L.figaro_batch_create(ctypes.byref(h), 0, None, 0) == 1
    inst = synth.two_relation(1, 50, 40, 2, 2, 5)
    p = F.Plan(inst.rels, analyze_only=True)
    arr = (ctypes.c_void_p * 1)(p._handle.value)
    assert L.figaro_batch_create(ctypes.byref(h), 1, arr, 0) == 1      # analyze-only plan
    assert b"analyze-only" in L.figaro_last_error(None)
    arr2 = (ctypes.c_void_p * 2)(p._handle.value, None)
    assert L.figaro_batch_create(ctypes.byref(h), 2, arr2, 0) == 1     # NULL plan


def test_tsqr_workspace_is_bounded_and_checked():
    """figaro_tsqr: workspace sizes stay within 8 MiB for any input, and bad
    arguments are rejected before anything is launched."""
    L = F.lib()
    for n in (1, 7, 16, 17, 32, 40, 41, 64, 100, 128):
        for rows in (0, 1, 100, 10**4, 10**6, 10**8, 10**11):
            b = L.figaro_tsqr_workspace_bytes(rows, n)
            assert 0 <= b <= 8 << 20, (n, rows, b)
        assert L.figaro_tsqr_workspace_bytes(10**6, n) > 0
    assert L.figaro_tsqr_workspace_bytes(100, 0) == -1
    assert L.figaro_tsqr_workspace_bytes(100, 129) == -1
    dummy = ctypes.c_void_p(0x1000)
    # unsupported width, negative rows, small leading dimension, missing or
    # short workspace
    assert L.figaro_tsqr(100, 129, dummy, 100, dummy, dummy, 1 << 30, None) == 9
    assert L.figaro_tsqr(-1, 8, dummy, 100, dummy, dummy, 1 << 30, None) == 1
    assert L.figaro_tsqr(100, 8, dummy, 99, dummy, dummy, 1 << 30, None) == 1
    need = L.figaro_tsqr_workspace_bytes(10**6, 8)
    assert L.figaro_tsqr(10**6, 8, dummy, 10**6, dummy, None, need, None) == 1
    assert L.figaro_tsqr(10**6, 8, dummy, 10**6, dummy, dummy, need - 8, None) == 1
    assert b"workspace" in L.figaro_last_error(None)
