"""The C-ABI library loads and exports every function include/msp.h declares
(no compute: runs without a GPU)."""
import ctypes

import pytest

import paper_2509_26193_amd as msp
from paper_2509_26193_amd import _lib


def test_library_exports_every_declared_symbol():
    names = msp.header_functions()
    assert "msp_find_targets" in names and "msp_commit_synapses" in names
    L = ctypes.CDLL(_lib.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name
    # the binding declares a signature for every exported function
    assert set(names) <= set(_lib._SIGS)


def test_status_strings():
    assert msp.status_string(0) == "ok"
    assert "capacity" in msp.status_string(-4)
    assert msp.status_string(12345) == "unknown status"


def test_invalid_handles_rejected_without_device():
    L = msp.lib()
    assert L.msp_update_vacant_counts(None, None, None, None) == _lib.MSP_ERR_INVALID
    assert L.msp_octree_info(None, None, None) == _lib.MSP_ERR_INVALID
    bm = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    h = ctypes.c_void_p()
    # n < 1, leaf_size != 1, bad box: rejected before any device call
    assert L.msp_build_octree(None, 0, bm, 1.0, 1, None, ctypes.byref(h)) == _lib.MSP_ERR_INVALID
    assert L.msp_build_octree(ctypes.c_void_p(8), 10, bm, 1.0, 2, None, ctypes.byref(h)) == _lib.MSP_ERR_INVALID
    assert L.msp_build_octree(ctypes.c_void_p(8), 10, bm, -1.0, 1, None, ctypes.byref(h)) == _lib.MSP_ERR_INVALID
    assert L.msp_build_octree(ctypes.c_void_p(8), 10, bm, float("nan"), 1, None, ctypes.byref(h)) == _lib.MSP_ERR_INVALID


def test_activity_arguments_rejected_without_device():
    L = msp.lib()
    P = _lib.ActivityParams(*[_lib.ACTIVITY[f] for f, _ in _lib.ActivityParams._fields_])
    p8 = ctypes.c_void_p(8)
    args = [p8, None, 0, None, None, None, 0, ctypes.byref(P), 1, 0, 1, p8, p8, p8, p8, p8, p8,
            None, None, None]
    assert L.msp_activity_run(0, *args) == _lib.MSP_ERR_INVALID          # n < 1
    bad = list(args)
    bad[6] = 3                                                          # approx outside 0..2
    assert L.msp_activity_run(10, *bad) == _lib.MSP_ERR_INVALID
    bad = list(args)
    bad[6] = 1                                                          # approx 1 needs ranks
    assert L.msp_activity_run(10, *bad) == _lib.MSP_ERR_INVALID
    Q = _lib.ActivityParams(*[_lib.ACTIVITY[f] for f, _ in _lib.ActivityParams._fields_])
    Q.epoch = 0
    bad = list(args)
    bad[7] = ctypes.byref(Q)                                            # epoch < 1
    assert L.msp_activity_run(10, *bad) == _lib.MSP_ERR_INVALID
    bad = list(args)
    bad[11] = None                                                      # no v
    assert L.msp_activity_run(10, *bad) == _lib.MSP_ERR_INVALID
