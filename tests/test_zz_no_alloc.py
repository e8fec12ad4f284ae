"""The allocation-free search (msp_find_targets_noalloc, for callers that cannot
allocate device memory) through the C ABI against msp_find_targets on the same
inputs: bitwise equal targets and offsets, on two calls in a row (the second smaller,
so it must not see the first call's leftovers in the shared fixed array), then the
size limit and the first call repeated."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2509_26193_amd as msp
from paper_2509_26193_amd import _lib
from synth_inputs import uniform_cube
from gpu_util import DEV, T, say

pytestmark = pytest.mark.gpu


def _tree(w):
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    msp.update_vacant_counts(tree, T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32))
    return tree, T(w.neuron_type, torch.uint8), T(w.vac_axon, torch.int32)


def _noalloc(L, tree, ty, va, w, seed, step):
    st = torch.cuda.current_stream().cuda_stream
    tgt = torch.full((max(w.searches, 1),), -7, dtype=torch.int32, device=DEV)
    off = torch.full((w.n + 1,), -7, dtype=torch.int64, device=DEV)
    rc = L.msp_find_targets_noalloc(tree.handle, ty.data_ptr(), va.data_ptr(), w.sigma, w.theta,
                                    seed, step, tgt.data_ptr(), off.data_ptr(), tgt.numel(), st)
    torch.cuda.synchronize()
    return rc, tgt[:w.searches].cpu().numpy(), off.cpu().numpy()


def _reference(L, tree, ty, va, w, seed, step):
    st = torch.cuda.current_stream().cuda_stream
    tgt = torch.full((max(w.searches, 1),), -9, dtype=torch.int32, device=DEV)
    off = torch.empty(w.n + 1, dtype=torch.int64, device=DEV)
    rc = L.msp_find_targets(tree.handle, ty.data_ptr(), va.data_ptr(), w.sigma, w.theta, seed,
                            step, tgt.data_ptr(), off.data_ptr(), tgt.numel(), st)
    torch.cuda.synchronize()
    assert rc == _lib.MSP_OK
    return tgt[:w.searches].cpu().numpy(), off.cpu().numpy()


def test_noalloc_search_equals_plain_search():
    L = msp.lib()
    big = uniform_cube(_lib.MSP_NOALLOC_MAX_NEURONS, 2000.0, seed=61)
    small = uniform_cube(3000, 700.0, seed=62)
    cases = [(big, 5, 0), (small, 6, 3)]
    trees = [_tree(w) for w, _, _ in cases]
    # the two allocation-free calls in a row, the second smaller
    got = []
    for (w, seed, step), (tree, ty, va) in zip(cases, trees):
        say(f"noalloc search n={w.n} searches={w.searches}")
        rc, tgt, off = _noalloc(L, tree, ty, va, w, seed, step)
        assert rc == _lib.MSP_OK, msp.status_string(rc)
        got.append((tgt, off))
    for k, ((w, seed, step), (tree, ty, va)) in enumerate(zip(cases, trees)):
        rt, ro = _reference(L, tree, ty, va, w, seed, step)
        assert np.array_equal(got[k][1], ro), k
        assert np.array_equal(got[k][0], rt), k
        assert not np.any(got[k][0] == -7)
    # beyond the fixed array: rejected before anything is queued
    w = uniform_cube(_lib.MSP_NOALLOC_MAX_NEURONS + 1, 2000.0, seed=63)
    tree, ty, va = _tree(w)
    rc, tgt, off = _noalloc(L, tree, ty, va, w, 1, 0)
    assert rc == _lib.MSP_ERR_TOO_LARGE
    assert np.all(tgt == -7) and np.all(off == -7)
    tree.free()
    # the first case again, after the smaller one: unchanged
    (w, seed, step), (tree, ty, va) = cases[0], trees[0]
    rc, tgt, off = _noalloc(L, tree, ty, va, w, seed, step)
    assert rc == _lib.MSP_OK and np.array_equal(tgt, got[0][0])
    for tree, _, _ in trees:
        tree.free()
    say("allocation-free search equals msp_find_targets")
