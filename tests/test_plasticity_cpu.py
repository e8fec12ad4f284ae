"""The 100-update workload on the oracle path: host-side element growth and synapse
deletion between connectivity updates (Sec. III-A, update of synaptic elements and
update of synapses), its bookkeeping invariants, and the resume pin: K updates in one
run equal K/2 updates, a save and reload of the state, and K/2 more, bitwise."""
import numpy as np

from oracle import oracle as orc
from synth_inputs import (PlasticityState, plasticity_init, plasticity_record, plasticity_step,
                          uniform_cube)


def _check_books(state: PlasticityState):
    n = state.z.shape[1]
    assert np.all(state.bound >= 0)
    assert np.array_equal(state.bound[0], np.bincount(state.syn_src, minlength=n))
    assert np.array_equal(state.bound[1], np.bincount(state.syn_tgt[state.syn_type == 0], minlength=n))
    assert np.array_equal(state.bound[2], np.bincount(state.syn_tgt[state.syn_type == 1], minlength=n))


def _updates(w, tree, state, vac, steps):
    """Connectivity updates on the oracle with the host plasticity in between."""
    formed = []
    for step in steps:
        a, e, i = vac
        tree.update_counts(e, i)
        off, src, elem = orc.search_list(a)
        o = tree.find_targets(w.neuron_type, w.sigma, w.theta, w.seed, step, src, elem)
        c = orc.commit(off, o["target"], w.neuron_type, a, e, i, w.seed, step)
        plasticity_record(state, c["syn_src"], c["syn_tgt"], c["syn_type"])
        _check_books(state)
        # the commit's decremented counts are the vacancies the books imply
        free = np.floor(state.z).astype(np.int64) - state.bound
        assert np.array_equal(c["vac_axon"], free[0])
        assert np.array_equal(c["vac_exc"], free[1])
        assert np.array_equal(c["vac_inh"], free[2])
        formed.append(c["n_formed"])
        vac = plasticity_step(state, w.neuron_type, w.seed, step)
        _check_books(state)
        assert np.all(state.bound <= np.floor(state.z))     # retraction broke enough synapses
        assert all(np.all(v >= 0) for v in vac)
    return vac, formed


def _workload():
    # the density of 8,388,608 neurons in a 20,000 um cube
    n = 3000
    edge = 20000.0 * (n / float(1 << 23)) ** (1.0 / 3.0)
    return uniform_cube(n, edge, seed=5)


def test_plasticity_bookkeeping_and_growth_rule_signs():
    w = _workload()
    state = plasticity_init(w)
    tree = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    vac, formed = _updates(w, tree, state, (w.vac_axon, w.vac_exc, w.vac_inh), range(6))
    assert formed[0] > 0 and state.syn_src.size > 0
    # synapses never link a neuron to itself (the source's own leaf is excluded)
    assert not np.any(state.syn_src == state.syn_tgt)
    # the growth rule: calcium at the target (0.7) neither grows nor retracts, below
    # the onset (0.4) retracts, in between grows
    from synth_inputs import growth_delta
    assert abs(growth_delta(np.array([0.7]))[0]) < 1e-12
    assert growth_delta(np.array([0.3]))[0] < 0 < growth_delta(np.array([0.55]))[0]


def test_resume_is_bitwise(tmp_path):
    w = _workload()
    tree = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    v0 = (w.vac_axon, w.vac_exc, w.vac_inh)
    s_full = plasticity_init(w)
    vac_full, _ = _updates(w, tree, s_full, v0, range(6))

    s_half = plasticity_init(w)
    vac_half, _ = _updates(w, tree, s_half, v0, range(3))
    s_half.save(tmp_path / "state.npz")
    np.savez(tmp_path / "vac.npz", *vac_half)
    s_res = PlasticityState.load(tmp_path / "state.npz")
    with np.load(tmp_path / "vac.npz") as f:
        vac_res = (f["arr_0"], f["arr_1"], f["arr_2"])
    vac_end, _ = _updates(w, tree, s_res, vac_res, range(3, 6))

    for a, b in zip(vac_full, vac_end):
        assert np.array_equal(a, b)
    assert np.array_equal(s_full.syn_src, s_res.syn_src)
    assert np.array_equal(s_full.syn_tgt, s_res.syn_tgt)
    assert np.array_equal(s_full.syn_type, s_res.syn_type)
    assert np.array_equal(s_full.z, s_res.z)
