"""The multi-update workload on the oracle path: connectivity updates with the
oracle's plasticity step in between (Sec. III-A, update of synaptic elements and
update of synapses), its bookkeeping invariants, and the resume pin: K updates in one
run equal K/2 updates, a save and reload of the state, and K/2 more, bitwise."""
import numpy as np

from oracle import oracle as orc
from synth_inputs import uniform_cube


def _check_books(net):
    src, tgt, ty = net.synapses()
    n = net.n
    assert np.all(net.bound >= 0)
    assert np.array_equal(net.bound[0], np.bincount(src, minlength=n))
    assert np.array_equal(net.bound[1], np.bincount(tgt[ty == 0], minlength=n))
    assert np.array_equal(net.bound[2], np.bincount(tgt[ty == 1], minlength=n))


def _updates(w, tree, net, vac, steps):
    """Connectivity updates on the oracle with its plasticity step in between."""
    formed = []
    for step in steps:
        a, e, i = vac
        tree.update_counts(e, i)
        off, src, elem = orc.search_list(a)
        o = tree.find_targets(w.neuron_type, w.sigma, w.theta, w.seed, step, src, elem)
        c = orc.commit(off, o["target"], w.neuron_type, a, e, i, w.seed, step)
        net.record(c["syn_src"], c["syn_tgt"], c["syn_type"])
        _check_books(net)
        # the commit's decremented counts are the vacancies the books imply
        free = np.floor(net.z).astype(np.int64) - net.bound
        assert np.array_equal(c["vac_axon"], free[0])
        assert np.array_equal(c["vac_exc"], free[1])
        assert np.array_equal(c["vac_inh"], free[2])
        formed.append(c["n_formed"])
        vac = net.step(w.seed, step)
        _check_books(net)
        assert np.all(net.bound <= np.floor(net.z))
        assert all(np.all(v >= 0) for v in vac)
    return vac, formed


def _workload():
    # the density of 8,388,608 neurons in a 20,000 um cube
    n = 3000
    edge = 20000.0 * (n / float(1 << 23)) ** (1.0 / 3.0)
    return uniform_cube(n, edge, seed=5)


def test_multi_update_bookkeeping():
    w = _workload()
    net = orc.Network(w.vac_axon, w.vac_exc, w.vac_inh, capacity=100000)
    tree = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    vac, formed = _updates(w, tree, net, (w.vac_axon, w.vac_exc, w.vac_inh), range(6))
    assert formed[0] > 0 and net.m > 0
    # synapses never link a neuron to itself (the source's own leaf is excluded)
    src, tgt, _ = net.synapses()
    assert not np.any(src == tgt)


def test_resume_is_bitwise(tmp_path):
    w = _workload()
    tree = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    v0 = (w.vac_axon, w.vac_exc, w.vac_inh)
    full = orc.Network(*v0, capacity=100000)
    vac_full, _ = _updates(w, tree, full, v0, range(6))

    half = orc.Network(*v0, capacity=100000)
    vac_half, _ = _updates(w, tree, half, v0, range(3))
    np.savez(tmp_path / "state.npz", z=half.z, bound=half.bound, src=half.src, tgt=half.tgt,
             type=half.type, m=half.m, a=vac_half[0], e=vac_half[1], i=vac_half[2])
    res = orc.Network(*v0, capacity=100000)
    with np.load(tmp_path / "state.npz") as f:
        res.z[:] = f["z"]
        res.bound[:] = f["bound"]
        res.src[:] = f["src"]
        res.tgt[:] = f["tgt"]
        res.type[:] = f["type"]
        res.m = int(f["m"])
        vac_res = (f["a"], f["e"], f["i"])
    vac_end, _ = _updates(w, tree, res, vac_res, range(3, 6))

    for a, b in zip(vac_full, vac_end):
        assert np.array_equal(a, b)
    for a, b in zip(full.synapses(), res.synapses()):
        assert np.array_equal(a, b)
    assert np.array_equal(full.z, res.z)
