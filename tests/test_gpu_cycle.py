"""The update cycle (msp_cycle_*): whole connectivity updates enqueued with every count
on the device (refresh, search, commit, record, plasticity step; Sec. III-A), eagerly
and as a replayed HIP graph. Its network state must equal, bitwise and after every
update, that of the same updates made of the separate calls, which the plasticity
tests check against the oracle."""
import numpy as np
import pytest
import torch

import paper_2509_26193_amd as msp
from synth_inputs import config_large, uniform_cube
from gpu_util import T, say

pytestmark = pytest.mark.gpu


def _workload(n, seed):
    edge = 20000.0 * (n / float(1 << 23)) ** (1.0 / 3.0)      # the 8M workload's density
    return uniform_cube(n, edge, seed=seed)


def _separate_update(tree, w, ty, net, vac, step):
    """One update made of the separate calls; returns the next vacancies."""
    ga, ge, gi = vac
    msp.update_vacant_counts(tree, ge, gi)
    tgt, off = msp.find_targets(tree, ty, ga, w.sigma, w.theta, w.seed, step)
    res = msp.commit_synapses(tgt, off, ty, ga, ge, gi, w.seed, step)
    net.record(res["syn_src"], res["syn_tgt"], res["syn_type"])
    return net.step(w.seed, step), int(off[-1].item()), int(res["n_formed"])


def _state(net, vac, m):
    torch.cuda.synchronize()
    return dict(z=net.z.cpu().numpy().copy(), bound=net.bound.cpu().numpy().copy(),
                src=net.src[:m].cpu().numpy().copy(), tgt=net.tgt[:m].cpu().numpy().copy(),
                type=net.type[:m].cpu().numpy().copy(), m=m,
                vac=[v.cpu().numpy().copy() for v in vac])


def _assert_same(a, b, label):
    assert a["m"] == b["m"], (label, a["m"], b["m"])
    for k in ("bound", "src", "tgt", "type"):
        assert np.array_equal(a[k], b[k]), (label, k)
    assert np.array_equal(a["z"].view(np.int64), b["z"].view(np.int64)), (label, "z")
    for x, y in zip(a["vac"], b["vac"]):
        assert np.array_equal(x, y), (label, "vacancies")


def _networks(w, cap):
    v0 = [T(v, torch.int32) for v in (w.vac_axon, w.vac_exc, w.vac_inh)]
    return msp.Network(*v0, capacity=cap), v0


def _compare_loops(w, updates, graph, cap, eager_work=False, label=""):
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    ty = T(w.neuron_type, torch.uint8)
    net_a, vac_a = _networks(w, cap)
    net_b, vac_b = _networks(w, cap)
    cyc = msp.Cycle(tree, ty, net_b, *vac_b, w.sigma, w.theta, w.seed, step=0, graph=graph)
    for step in range(updates):
        vac_a, S, formed = _separate_update(tree, w, ty, net_a, vac_a, step)
        ref = _state(net_a, vac_a, net_a.m)
        if eager_work:                  # unrelated device work between replays
            x = torch.randn(1 << 20, device="cuda:0")
            float((x * 3.0).sum())
        cyc.run(1)
        c = cyc.counts()
        assert cyc.status() == 0, cyc.status()
        assert c["step"] == step + 1 and c["searches"] == S and c["formed"] == formed, (c, S, formed)
        _assert_same(_state(net_b, cyc.va_ve_vi(), c["m"]), ref, f"{label} update {step}")
        say(f"[{label}] update {step}: {S} searches, {formed} formed, {c['m']} synapses: equal")
    cyc.free()
    tree.free()


def test_cycle_equals_separate_calls_65536():
    _compare_loops(_workload(65536, 11), 6, graph=False, cap=1_000_000, label="eager")


def test_cycle_graph_replays_equal_separate_calls_65536():
    _compare_loops(_workload(65536, 12), 6, graph=True, cap=1_000_000, eager_work=True,
                   label="graph")


def test_cycle_graph_8388608_three_updates():
    """The 2^23-neuron workload the benchmark loops over: three replayed updates, each
    equal to the separate calls bitwise."""
    w = config_large()
    _compare_loops(w, 3, graph=True, cap=4 * w.n, label="8M graph")


def test_cycle_many_updates_in_one_run():
    """Several updates enqueued by one call (the host reads nothing in between)."""
    w = _workload(32768, 13)
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    ty = T(w.neuron_type, torch.uint8)
    net_a, vac_a = _networks(w, 500_000)
    net_b, vac_b = _networks(w, 500_000)
    for step in range(5):
        vac_a, _, _ = _separate_update(tree, w, ty, net_a, vac_a, step)
    ref = _state(net_a, vac_a, net_a.m)
    cyc = msp.Cycle(tree, ty, net_b, *vac_b, w.sigma, w.theta, w.seed, step=0, graph=True)
    cyc.run(2)
    cyc.run(3)
    c = cyc.counts()
    assert cyc.status() == 0 and c["step"] == 5
    _assert_same(_state(net_b, cyc.va_ve_vi(), c["m"]), ref, "5 updates")
    cyc.free()
    tree.free()


def test_cycle_capacity_errors_are_reported_not_written():
    w = _workload(16384, 14)
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    ty = T(w.neuron_type, torch.uint8)
    S0 = int(w.vac_axon.sum())
    # too few search slots: the update searches and forms nothing, the step still runs
    net, vac = _networks(w, 200_000)
    cyc = msp.Cycle(tree, ty, net, *vac, w.sigma, w.theta, w.seed, search_capacity=S0 - 1,
                    graph=True)
    cyc.run(1)
    c = cyc.counts()
    assert cyc.status() == msp._lib.MSP_CYCLE_SEARCH_CAPACITY
    assert c["searches"] == 0 and c["formed"] == 0 and c["m"] == 0 and c["step"] == 1
    assert int(net.bound.sum().item()) == 0
    cyc.free()
    # a synapse list too short for the first update's synapses: none recorded
    net, vac = _networks(w, 10)
    cyc = msp.Cycle(tree, ty, net, *vac, w.sigma, w.theta, w.seed, graph=False)
    cyc.run(1)
    c = cyc.counts()
    assert cyc.status() == msp._lib.MSP_CYCLE_SYN_CAPACITY
    assert c["formed"] > 10 and c["m"] == 0
    assert int(net.bound.sum().item()) == 0
    cyc.free()
    tree.free()
