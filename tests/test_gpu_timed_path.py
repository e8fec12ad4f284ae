"""The search instance the benchmark times (no diagnostics: no per-search counters,
the launch shape of msp_find_targets) against the oracle at the benchmarked sizes,
and the handle lifetime and the smaller entry points of the C ABI on the device.

Any diagnostic output switches the search to its counting instantiation (another
kernel, another occupancy, other checkpoint intervals). Here the targets of the plain
call are compared bitwise with those of a counting call, and a sample of at least
65,536 searches of the plain call with the oracle (Sec. III-B, "Division of work": the
accepted list, the draw and the restart), with the counting call's normalisers."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2509_26193_amd as msp
from oracle import oracle as orc
from synth_inputs import config_clusters, config_large, uniform_cube
from gpu_util import DEV, T, compare_search, oracle_tree, say

pytestmark = pytest.mark.gpu

SAMPLE = 65536


def _timed_against_oracle(w, label, seed=5):
    say(f"[{label}] n={w.n} searches={w.searches} theta={w.theta}")
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    msp.update_vacant_counts(tree, T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32))
    ty, va = T(w.neuron_type, torch.uint8), T(w.vac_axon, torch.int32)
    buf = torch.full((w.searches,), -7, dtype=torch.int32, device=DEV)
    # the benchmark's call: preallocated output, no diagnostics
    tgt, off = msp.find_targets(tree, ty, va, w.sigma, w.theta, w.seed, w.step, target_out=buf)
    torch.cuda.synchronize()
    timed = tgt.cpu().numpy().astype(np.int64)
    assert timed.size == w.searches and not np.any(timed == -7)
    # a counting call on the same tree: same targets, and its normalisers
    tgt2, _, z0, _, _ = msp.find_targets(tree, ty, va, w.sigma, w.theta, w.seed, w.step,
                                         diag=True, counters=True)
    torch.cuda.synchronize()
    assert np.array_equal(timed, tgt2.cpu().numpy().astype(np.int64)), label
    z0 = z0.cpu().numpy()
    tree.free()
    t = oracle_tree(w)
    ooff, src, elem = orc.search_list(w.vac_axon)
    assert np.array_equal(off.cpu().numpy(), ooff)
    q = np.sort(np.random.default_rng(seed).choice(src.size, size=min(SAMPLE, src.size),
                                                   replace=False))
    o = t.find_targets(w.neuron_type, w.sigma, w.theta, w.seed, w.step, src[q], elem[q])
    compare_search(timed[q], z0[q], o, f"{label} timed instance, {q.size} sampled")
    del t


def test_timed_search_8388608_uniform():
    _timed_against_oracle(config_large(), "8M uniform")


def test_timed_search_1048576_clusters_theta03():
    _timed_against_oracle(config_clusters(theta=0.3), "1M clusters theta 0.3")


def test_handles_and_small_entry_points():
    L = msp.lib()
    st = torch.cuda.current_stream().cuda_stream
    w = uniform_cube(20000, 1500.0, seed=17)
    ty, va = T(w.neuron_type, torch.uint8), T(w.vac_axon, torch.int32)
    ve, vi = T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32)
    # search offsets: the CSR prefix sum and the number of searches
    off, S = msp.search_offsets(va)
    torch.cuda.synchronize()
    ref = np.concatenate([[0], np.cumsum(w.vac_axon.astype(np.int64))])
    assert S == w.searches and np.array_equal(off.cpu().numpy(), ref)
    bad = va.clone()
    bad[5] = -1
    with pytest.raises(msp.MspError):
        msp.search_offsets(bad)
    # a search after the workspace was released equals one before
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    msp.update_vacant_counts(tree, ve, vi)
    a, _ = msp.find_targets(tree, ty, va, w.sigma, w.theta, 3, 1)
    a = a.cpu().numpy()
    msp.release_workspace()
    msp.release_workspace()                          # nothing held: still fine
    b, _ = msp.find_targets(tree, ty, va, w.sigma, w.theta, 3, 1)
    assert np.array_equal(a, b.cpu().numpy())
    # a freed handle is rejected by every call; freeing twice does nothing
    h = tree.handle
    assert L.msp_free_octree_async(h, st) == msp._lib.MSP_OK
    tree._h = None
    n_nodes = ctypes.c_int64()
    assert L.msp_octree_info(h, None, ctypes.byref(n_nodes)) == msp._lib.MSP_ERR_INVALID
    assert L.msp_update_vacant_counts(h, ve.data_ptr(), vi.data_ptr(), st) == msp._lib.MSP_ERR_INVALID
    assert L.msp_find_targets(h, ty.data_ptr(), va.data_ptr(), w.sigma, w.theta, 3, 1, None,
                              off.data_ptr(), 0, st) == msp._lib.MSP_ERR_INVALID
    assert L.msp_last_device_error(h) == msp._lib.MSP_ERR_INVALID
    assert L.msp_free_octree_async(h, st) == msp._lib.MSP_ERR_INVALID
    L.msp_free_octree(h)
    # the synchronous free, then the same checks
    t2 = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    h2 = t2.handle
    L.msp_free_octree(h2)
    t2._h = None
    assert L.msp_octree_info(h2, None, None) == msp._lib.MSP_ERR_INVALID
    L.msp_free_octree(h2)
    # the activity's initial state comes from the library: v = c, u = b c by type
    act = msp.Activity(ty)
    torch.cuda.synchronize()
    p = msp.ACTIVITY
    c = np.where(w.neuron_type == 1, p["c_inh"], p["c_exc"])
    b = np.where(w.neuron_type == 1, p["b_inh"], p["b_exc"])
    assert np.array_equal(act.v.cpu().numpy(), c)
    assert np.array_equal(act.u.cpu().numpy(), b * c)
    for x in (act.calcium, act.freq):
        assert not torch.any(x != 0)
    assert not torch.any(act.spiked != 0) and not torch.any(act.count != 0)
    say("handles, search offsets, workspace release and activity start: ok")
