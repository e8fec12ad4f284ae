"""The 100-update workload on the GPU: positions fixed, the octree built once, then per
update a vacancy refresh, the search and the commit on the device, with the host-side
element growth and synapse deletion in between (Sec. III-A). Every update is checked
against the oracle fed the same pre-update state; a resumed run equals an
uninterrupted one bitwise."""
import numpy as np
import pytest
import torch

import paper_2509_26193_amd as msp
from oracle import oracle as orc
from synth_inputs import (PlasticityState, config_large, plasticity_init, plasticity_record,
                          plasticity_step, uniform_cube)
from gpu_util import T, compare_search, say, MAX_DIFF_SHARE, WINDOW

pytestmark = pytest.mark.gpu


def _gpu_update(tree, w, ty, vac, step):
    """One connectivity update on the device. Returns host copies of everything."""
    ga, ge, gi = (T(v, torch.int32) for v in vac)
    msp.update_vacant_counts(tree, ge, gi)
    tgt, off, z0, _ = msp.find_targets(tree, ty, ga, w.sigma, w.theta, w.seed, step, diag=True)
    res = msp.commit_synapses(tgt, off, ty, ga, ge, gi, w.seed, step)
    torch.cuda.synchronize()
    return dict(target=tgt.cpu().numpy().astype(np.int64), off=off.cpu().numpy(),
                z0=z0.cpu().numpy(), syn_src=res["syn_src"].cpu().numpy(),
                syn_tgt=res["syn_tgt"].cpu().numpy(), syn_type=res["syn_type"].cpu().numpy(),
                vac=(ga.cpu().numpy(), ge.cpu().numpy(), gi.cpu().numpy()))


def _run(w, tree, ty, state, vac, steps, otree=None, label=""):
    lists = []
    for step in steps:
        g = _gpu_update(tree, w, ty, vac, step)
        if otree is not None:
            a, e, i = vac
            otree.update_counts(e, i)
            ooff, src, elem = orc.search_list(a)
            o = otree.find_targets(w.neuron_type, w.sigma, w.theta, w.seed, step, src, elem)
            compare_search(g["target"], g["z0"], o, f"{label} update {step}")
            oc = orc.commit(ooff, g["target"], w.neuron_type, a, e, i, w.seed, step)
            assert np.array_equal(g["syn_src"], oc["syn_src"])
            assert np.array_equal(g["syn_tgt"], oc["syn_tgt"])
            assert np.array_equal(g["syn_type"], oc["syn_type"])
            for x, y in zip(g["vac"], (oc["vac_axon"], oc["vac_exc"], oc["vac_inh"])):
                assert np.array_equal(x, y)
        lists.append((g["syn_src"], g["syn_tgt"], g["syn_type"]))
        plasticity_record(state, g["syn_src"], g["syn_tgt"], g["syn_type"])
        vac = plasticity_step(state, w.neuron_type, w.seed, step)
        say(f"[{label}] update {step}: {g['target'].size} searches, {g['syn_src'].size} formed, "
            f"{state.syn_src.size} synapses")
    return vac, lists


def test_updates_65536_full_oracle_and_resume(tmp_path):
    n = 65536
    edge = 20000.0 * (n / float(1 << 23)) ** (1.0 / 3.0)      # the 8M workload's density
    w = uniform_cube(n, edge, seed=11)
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    ty = T(w.neuron_type, torch.uint8)
    otree = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    v0 = (w.vac_axon, w.vac_exc, w.vac_inh)
    state = plasticity_init(w)
    vac4, first = _run(w, tree, ty, state, v0, range(4), otree, "65536")
    state.save(tmp_path / "state.npz")
    saved_vac = tuple(v.copy() for v in vac4)
    _, rest = _run(w, tree, ty, state, vac4, range(4, 8), otree, "65536")
    # resume from the saved state: the same lists, bitwise
    resumed = PlasticityState.load(tmp_path / "state.npz")
    _, again = _run(w, tree, ty, resumed, saved_vac, range(4, 8), None, "65536 resumed")
    for (a, b, c), (x, y, z) in zip(rest, again):
        assert np.array_equal(a, x) and np.array_equal(b, y) and np.array_equal(c, z)
    assert np.array_equal(resumed.syn_src, state.syn_src)
    tree.free()


def test_updates_8388608_sampled_oracle():
    w = config_large()
    say(f"8M workload: n={w.n}")
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    ty = T(w.neuron_type, torch.uint8)
    otree = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    state = plasticity_init(w)
    vac = (w.vac_axon, w.vac_exc, w.vac_inh)
    rng = np.random.default_rng(2024)
    for step in range(3):
        a, e, i = vac
        g = _gpu_update(tree, w, ty, vac, step)
        # the oracle on 65,536 sampled searches of this update
        otree.update_counts(e, i)
        ooff, src, elem = orc.search_list(a)
        pick = np.sort(rng.choice(src.size, size=min(65536, src.size), replace=False))
        o = otree.find_targets(w.neuron_type, w.sigma, w.theta, w.seed, step, src[pick], elem[pick])
        diff = g["target"][pick] != o["target"]
        outside = diff & ~(o["window"] < WINDOW)
        pos = o["z0"] > 0
        rel = np.abs(g["z0"][pick][pos] - o["z0"][pos]) / o["z0"][pos]
        say(f"[8M update {step}] searches={src.size} sampled={pick.size} differing={int(diff.sum())} "
            f"outside-window={int(outside.sum())} max-rel-z0={rel.max():.2e}")
        assert int(outside.sum()) == 0
        assert diff.mean() < MAX_DIFF_SHARE or int(diff.sum()) <= 1
        assert rel.max() < 1e-5
        # the commit of the GPU's proposals, bitwise against the oracle's commit
        oc = orc.commit(ooff, g["target"], w.neuron_type, a, e, i, w.seed, step)
        assert np.array_equal(g["syn_src"], oc["syn_src"])
        assert np.array_equal(g["syn_tgt"], oc["syn_tgt"])
        assert np.array_equal(g["syn_type"], oc["syn_type"])
        plasticity_record(state, g["syn_src"], g["syn_tgt"], g["syn_type"])
        vac = plasticity_step(state, w.neuron_type, w.seed, step)
        say(f"[8M update {step}] formed {g['syn_src'].size}, synapses {state.syn_src.size}")
    tree.free()
