"""The C ABI without a GPU: the library loads, exports every function that
include/sldg.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_1603_07008_amd as sl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sldg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sldg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(sl.LIB_PATH):
        from paper_1603_07008_amd import build
        build.build(force=False)
    return sl.lib()


def test_exports_every_declared_function(L):
    names = _declared()
    assert set(names) == set(sl.EXPORTS), names
    for n in names:
        assert hasattr(L, n), n


def _plan(L, ndim, ncells, k, tier):
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * max(1, len(ncells)))(*ncells) if ncells is not None else None
    return L.sldg_plan(ctypes.byref(h), ndim, arr, k, tier, None), h


def test_plan_rejects_bad_arguments_before_the_device(L):
    assert L.sldg_plan(None, 1, None, 2, 1, None) == sl.SLDG_ERR_ARG
    st, h = _plan(L, 0, [4], 2, 1)
    assert st == sl.SLDG_ERR_ARG and h.value is None
    st, _ = _plan(L, 7, [4] * 7, 2, 1)
    assert st == sl.SLDG_ERR_ARG
    st, _ = _plan(L, 1, None, 2, 1)
    assert st == sl.SLDG_ERR_ARG
    st, _ = _plan(L, 1, [4], 4, 1)
    assert st == sl.SLDG_ERR_UNSUPPORTED and "degree" in sl.last_error()
    st, _ = _plan(L, 1, [4], 0, 1)
    assert st == sl.SLDG_ERR_UNSUPPORTED
    st, _ = _plan(L, 1, [4], 2, 9)
    assert st == sl.SLDG_ERR_UNSUPPORTED
    st, _ = _plan(L, 2, [4, 0], 2, 1)
    assert st == sl.SLDG_ERR_ARG
    st, _ = _plan(L, 2, [1 << 16, 1 << 16], 2, 1)
    assert st == sl.SLDG_ERR_UNSUPPORTED


def test_calls_on_a_null_plan(L):
    assert L.sldg_advect_dim(None, 0, None, 0, None, None, None, None) == sl.SLDG_ERR_ARG
    out = (ctypes.c_double * 2)()
    assert L.sldg_mass(None, None, out) == sl.SLDG_ERR_ARG
    assert L.sldg_split_steps(None, None, 0, 0, None, None, None, None, None) == sl.SLDG_ERR_ARG
    assert L.sldg_line_tables(None, 0, 1, None, None, None) == sl.SLDG_ERR_ARG
    assert L.sldg_plan_set_stream(None, None) == sl.SLDG_ERR_ARG
    assert L.sldg_timing_enable(None, 1) == sl.SLDG_ERR_ARG
    assert L.sldg_mass_device(None, None, None) == sl.SLDG_ERR_ARG
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    assert L.sldg_timing_read(None, 0, ctypes.byref(n), ctypes.byref(ms)) == sl.SLDG_ERR_ARG
    # copy: argument checks happen before any device call
    assert L.sldg_device_copy(None, None, 16, None) == sl.SLDG_ERR_ARG
    assert L.sldg_device_copy(16, 64, 15, None) == sl.SLDG_ERR_ARG
    assert L.sldg_device_copy(16, 40, 16, None) == sl.SLDG_ERR_ARG
    assert L.sldg_device_copy(16, 32, 32, None) == sl.SLDG_ERR_ALIAS
    assert L.sldg_hi_bytes(None) == -1
    f = ctypes.c_int(-1)
    assert L.sldg_plan_sweep_form(None, 1, 0, None, None, None, None, ctypes.byref(f)) == \
        sl.SLDG_ERR_ARG and f.value == -1
    L.sldg_plan_destroy(None)


def test_status_strings(L):
    for st in range(6):
        assert sl.status_string(st)
    assert sl.status_string(99) == "unknown status"


def test_batch_rejects_bad_arguments_before_the_device(L):
    from paper_1603_07008_amd import batch as B
    BL = B._lib()
    h = ctypes.c_void_p()
    n = (ctypes.c_int64 * 4)(8, 8, 8, 8)
    k = (ctypes.c_int * 2)(2, 2)
    assert BL.sldg_batch_create(None, 2, 2, n, k, 1, None) == sl.SLDG_ERR_ARG
    assert BL.sldg_batch_create(ctypes.byref(h), 0, 2, n, k, 1, None) == sl.SLDG_ERR_ARG
    assert BL.sldg_batch_create(ctypes.byref(h), 2, 9, n, k, 1, None) == sl.SLDG_ERR_ARG
    assert BL.sldg_batch_create(ctypes.byref(h), 2, 2, n, k, 7, None) == sl.SLDG_ERR_UNSUPPORTED
    kbad = (ctypes.c_int * 2)(2, 5)
    assert BL.sldg_batch_create(ctypes.byref(h), 2, 2, n, kbad, 1, None) == sl.SLDG_ERR_UNSUPPORTED
    nbad = (ctypes.c_int64 * 4)(8, 0, 8, 8)
    assert BL.sldg_batch_create(ctypes.byref(h), 2, 2, nbad, k, 1, None) == sl.SLDG_ERR_ARG
    assert BL.sldg_batch_run(None, 1, 0, None) == sl.SLDG_ERR_ARG
    assert BL.sldg_batch_tune(None, 1) == sl.SLDG_ERR_ARG
    BL.sldg_batch_destroy(None)


def test_tuner_candidates_are_valid_shapes(L):
    """The autotuner's candidate lists (host data, no device): every shape is
    one sldg_plan_set_shape accepts, the dimension-0 list offers the group
    (rows 4) and lane (rows 1) forms with the same tuple counts, and the
    strided list offers the lane form (rows 0) beside 2, 4 and 8 rows."""
    def cands(strided):
        out, i = [], 0
        while True:
            r, t, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            st = L.sldg_tune_candidate(strided, i, ctypes.byref(r), ctypes.byref(t), ctypes.byref(c))
            if st != 0:
                assert st == sl.SLDG_ERR_ARG
                return out
            out.append((r.value, t.value, c.value))
            i += 1
    contig, strided = cands(0), cands(1)
    assert {r for r, _, _ in contig} == {1, 4}
    assert {t for r, t, _ in contig if r == 1} == {t for r, t, _ in contig if r == 4}
    assert {r for r, _, _ in strided} == {0, 2, 4, 8}
    assert all(c in (1, 2, 4) and t >= 0 for _, t, c in contig)
    flags = sl.SLDG_SHAPE_STAGED | sl.SLDG_SHAPE_MEMORDER
    assert all(c & ~flags in (1, 2, 4) and t >= 0 for _, t, c in strided)
    staged = [(r, c) for r, _, c in strided if c & sl.SLDG_SHAPE_STAGED]
    assert staged and all(r in (4, 8) for r, _ in staged)
    memorder = [(r, c) for r, _, c in strided if c & sl.SLDG_SHAPE_MEMORDER]
    assert memorder and all(r > 0 for r, _ in memorder)
    assert len(set(strided)) == len(strided) and len(set(contig)) == len(contig)


def test_allocation_limit_forces_nomem_before_the_device(L):
    """sldg_set_device_alloc_limit: a plan whose tables pass the cap is
    refused with SLDG_ERR_NOMEM before any device call (so on a machine
    without a GPU too); removing the cap restores the normal path."""
    assert L.sldg_set_device_alloc_limit(-2) == sl.SLDG_ERR_ARG
    assert L.sldg_set_device_alloc_limit(0) == sl.SLDG_OK
    try:
        held = L.sldg_device_alloc_bytes()
        st, h = _plan(L, 2, [16, 16], 2, 1)
        assert st == sl.SLDG_ERR_NOMEM and h.value is None
        assert "allocation limit" in sl.last_error()
        assert L.sldg_device_alloc_bytes() == held
    finally:
        assert L.sldg_set_device_alloc_limit(-1) == sl.SLDG_OK
    st, h = _plan(L, 2, [16, 16], 2, 1)
    assert st != sl.SLDG_ERR_NOMEM
    if st == sl.SLDG_OK:
        L.sldg_plan_destroy(h)
