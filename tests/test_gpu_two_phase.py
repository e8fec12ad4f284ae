"""The two-phase (location-aware) search of Sec. IV-A on one GPU: restarts from a drawn
cell at or below the branch level become requests that a second pass runs in cell
order. The paper's change moves where a restart is computed, not what it computes, so
the targets and every per-search count must equal the one-phase search's bitwise, for
every branch level; the request count must equal the number of chains that reach a
cell that deep (all restarts at level 1)."""
import numpy as np
import pytest
import torch

import paper_2509_26193_amd as msp
from oracle import oracle as orc
from synth_inputs import config_clusters, config_large, uniform_cube
from gpu_util import T, compare_search, oracle_tree, say

pytestmark = pytest.mark.gpu

LEVELS = (1, 2, 4, 6, 9, 21)


def _run(tree, w, ty, va, branch_level):
    info = {}
    tgt, off, z0, lv, cnt = msp.find_targets(tree, ty, va, w.sigma, w.theta, w.seed, w.step,
                                             diag=True, counters=True,
                                             branch_level=branch_level, phase2=info)
    torch.cuda.synchronize()
    out = dict(target=tgt.cpu().numpy(), z0=z0.cpu().numpy(), levels=lv.cpu().numpy(),
               off=off.cpu().numpy(), requests=info["requests"])
    for k in ("visits", "opens", "visits0", "opens0"):
        out[k] = cnt[k].cpu().numpy()
    return out


def _check_levels(w, label, levels=LEVELS):
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    msp.update_vacant_counts(tree, T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32))
    ty, va = T(w.neuron_type, torch.uint8), T(w.vac_axon, torch.int32)
    one = _run(tree, w, ty, va, -1)
    assert one["requests"] == 0
    restarted = int((one["levels"] > 1).sum())
    prev = None
    for b in levels:
        two = _run(tree, w, ty, va, b)
        say(f"[{label}] branch level {b}: {two['requests']} second-phase requests "
            f"({restarted} searches restart)")
        for k in ("target", "z0", "levels", "visits", "opens", "visits0", "opens0"):
            assert np.array_equal(one[k], two[k]), (label, b, k)
        if b == 1:
            assert two["requests"] == restarted
        if prev is not None:
            assert two["requests"] <= prev
        prev = two["requests"]
    tree.free()
    return one


def test_two_phase_equals_one_phase_and_oracle():
    w = uniform_cube(65536, 20000.0 * (65536 / float(1 << 23)) ** (1.0 / 3.0), seed=21)
    one = _check_levels(w, "uniform 65536")
    t = oracle_tree(w)
    off, src, elem = orc.search_list(w.vac_axon)
    o = t.find_targets(w.neuron_type, w.sigma, w.theta, w.seed, w.step, src, elem)
    compare_search(one["target"].astype(np.int64), one["z0"], o, "two-phase 65536")


def test_two_phase_clusters():
    w = config_clusters()
    _check_levels(w, "clusters 1M", levels=(1, 5, 8))


def test_two_phase_8388608():
    w = config_large()
    _check_levels(w, "uniform 8M", levels=(1, 6))
