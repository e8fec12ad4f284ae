"""The level-0 walk cut into pre-order parts (a launch with few tiles walks each tile's
parts on different wavefronts) finds the same nodes as the whole walk: visits, opens,
levels and targets equal, z0 equal up to the rounding of adding the part sums. Checked
against the oracle as well, on a dense case, a sparse one (few sources over many
neurons, the case parts are for) and a clustered one."""
import numpy as np
import pytest
import torch

import paper_2509_26193_amd as msp
from gpu_util import T, compare_search, oracle_tree, say
from oracle import oracle as orc
from synth_inputs import config_clusters, uniform_cube

pytestmark = pytest.mark.gpu


def _run(tree, w, va, parts):
    ty = T(w.neuron_type, torch.uint8)
    tgt, off, z0, lv, cnt = msp.find_targets(tree, ty, va, w.sigma, w.theta, w.seed, w.step,
                                             diag=True, counters=True, parts=parts)
    torch.cuda.synchronize()
    out = dict(target=tgt.cpu().numpy().astype(np.int64), z0=z0.cpu().numpy(),
               levels=lv.cpu().numpy())
    out.update({k: v.cpu().numpy() for k, v in cnt.items() if k != "wave_steps"})
    return out


@pytest.mark.parametrize("case", ["dense", "sparse", "clusters"])
def test_parts_equal_whole_walk(case):
    if case == "clusters":
        w = config_clusters(seed=51, n_centres=8, per_centre=15000, edge=6000.0)
    else:
        w = uniform_cube(120000, 3000.0, seed=52)
    va_h = np.asarray(w.vac_axon).copy()
    if case == "sparse":                      # about 6 % of the neurons search
        keep = np.random.default_rng(53).random(va_h.size) < 0.06
        va_h = np.where(keep, va_h, 0).astype(np.int32)
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    msp.update_vacant_counts(tree, T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32))
    va = T(va_h, torch.int32)
    ref = _run(tree, w, va, 1)
    for parts in (0, 2, 4, 8):
        g = _run(tree, w, va, parts)
        for k in ("target", "levels", "visits", "opens", "visits0", "opens0"):
            assert np.array_equal(g[k], ref[k]), (case, parts, k)
        pos = ref["z0"] > 0
        assert np.array_equal(g["z0"] > 0, pos)
        rel = np.abs(g["z0"][pos] - ref["z0"][pos]) / ref["z0"][pos]
        assert rel.max(initial=0.0) < 1e-12, (case, parts, rel.max())
        say(f"{case}: {parts} parts per tile ({pos.sum()} searches) equal the whole walk, "
            f"max rel z0 {rel.max(initial=0.0):.1e}")
    # and the whole thing against the oracle
    off, src, elem = orc.search_list(va_h)
    o = oracle_tree(w).find_targets(w.neuron_type, w.sigma, w.theta, w.seed, w.step, src, elem)
    g = _run(tree, w, va, 8)
    compare_search(g["target"], g["z0"], o, f"{case} 8 parts")
    tree.free()


def test_parts_argument_checked():
    w = uniform_cube(5000, 1000.0, seed=54)
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    msp.update_vacant_counts(tree, T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32))
    with pytest.raises(Exception):
        msp.find_targets(tree, T(w.neuron_type, torch.uint8), T(w.vac_axon, torch.int32),
                         w.sigma, w.theta, w.seed, w.step, parts=3)
    tree.free()
