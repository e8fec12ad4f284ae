"""Batched search: one set of launches over many independent simulations must give,
per simulation, exactly the targets of the plain search with the same arguments,
including when replayed from a captured HIP graph."""
import numpy as np
import pytest
import torch

import paper_2509_26193_amd as msp
from oracle import oracle as orc
from synth_inputs import config_batched
from gpu_util import T, compare_search, compare_targets, say

pytestmark = pytest.mark.gpu


def _setup(n_sims=10, lo=10, hi=14, seed=3):
    ws = config_batched(seed=seed, n_sims=n_sims, log2_lo=lo, log2_hi=hi)
    sims = []
    for k, w in enumerate(ws):
        tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
        ve, vi = T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32)
        msp.update_vacant_counts(tree, ve, vi)
        sims.append(dict(tree=tree, neuron_type=T(w.neuron_type, torch.uint8),
                         vac_axon=T(w.vac_axon, torch.int32), sigma=w.sigma, seed=1000 + k))
    return ws, sims


def _plain(sims, theta, step):
    out = []
    for d in sims:
        tgt, off = msp.find_targets(d["tree"], d["neuron_type"], d["vac_axon"], d["sigma"], theta,
                                    d["seed"], step)
        out.append((tgt.cpu().numpy().copy(), off.cpu().numpy().copy()))
    return out


def _check_equal(batch, ref, label):
    torch.cuda.synchronize()
    assert batch.status() == [0] * batch.n_sims
    for k, (rt, ro) in enumerate(ref):
        tgt, off = batch.results(k)
        assert np.array_equal(off.cpu().numpy(), ro), (label, k)
        assert np.array_equal(tgt.cpu().numpy(), rt), (label, k)


def test_batched_equals_plain_and_oracle():
    ws, sims = _setup()
    say(f"batch of {len(ws)}: n = {[w.n for w in ws]}")
    ref = _plain(sims, 0.3, 7)
    b = msp.Batch(sims)
    b.run(0.3, 7)
    _check_equal(b, ref, "eager")
    # the small simulations against the oracle
    for k, w in enumerate(ws[:4]):
        t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
        t.update_counts(w.vac_exc, w.vac_inh)
        off, src, elem = orc.search_list(w.vac_axon)
        o = t.find_targets(w.neuron_type, w.sigma, 0.3, 1000 + k, 7, src, elem)
        tgt, _ = b.results(k)
        g = tgt.cpu().numpy().astype(np.int64)
        diff = g != o["target"]
        assert np.all(o["window"][diff] < 1e-6), k
    b.free()


def test_batched_graph_replays_match_eager():
    ws, sims = _setup(n_sims=6, seed=4)
    b = msp.Batch(sims, graph=True)
    other = sims[0]
    for rep, step in enumerate((3, 4, 3, 9)):
        ref = _plain(sims, 0.35, step)
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda:0")
        y = (x * 2.0).sum()
        msp.find_targets(other["tree"], other["neuron_type"], other["vac_axon"], 500.0, 0.5, 77, 1)
        torch.cuda.synchronize()
        b.run(0.35, step)
        _check_equal(b, ref, f"replay {rep} step {step}")
        say(f"replay {rep} (step {step}) ok, eager work value {float(y):.3f}")
    b.free()


def test_batched_autotune_and_new_buffers():
    ws, sims = _setup(n_sims=5, seed=6)
    ref = _plain(sims, 0.3, 2)
    b = msp.Batch(sims, graph=True, autotune=True)
    b.run(0.3, 2)
    _check_equal(b, ref, "autotuned")
    # new vacancy counts (same octrees): pass the new buffers on the next run
    for d in b.sims:
        d["vac_axon"] = torch.clamp(d["vac_axon"] - 1, min=0).contiguous()
        S = int(d["vac_axon"].sum().item())
        d["target_out"] = torch.empty(max(S, 1), dtype=torch.int32, device="cuda:0")
    ref2 = _plain(b.sims, 0.3, 5)
    b.run(0.3, 5, update=True)
    _check_equal(b, ref2, "new buffers")
    b.free()


def test_batched_capacity_error_is_per_simulation():
    ws, sims = _setup(n_sims=4, seed=8)
    ref = _plain(sims, 0.3, 1)
    sims[2] = dict(sims[2])
    sims[2]["target_out"] = torch.full((3,), -9, dtype=torch.int32, device="cuda:0")
    b = msp.Batch(sims)
    b.run(0.3, 1)
    st = b.status()
    assert st[2] == msp._lib.MSP_ERR_CAPACITY
    assert [st[k] for k in (0, 1, 3)] == [0, 0, 0]
    assert torch.all(b.sims[2]["target_out"] == -9)          # not written
    for k in (0, 1, 3):
        tgt, off = b.results(k)
        assert np.array_equal(tgt.cpu().numpy(), ref[k][0])
    b.free()


def test_config4_64_simulations_against_oracle():
    """The 64-simulation workload (2^12..2^18 neurons each, 4.0M in all) as the benchmark
    runs it (one autotuned, graph-captured batch): every search of the simulations with
    at most 2^14 neurons and 20,000 sampled searches of each larger one against the
    oracle."""
    ws = config_batched()
    sims = []
    for k, w in enumerate(ws):
        tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
        msp.update_vacant_counts(tree, T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32))
        sims.append(dict(tree=tree, neuron_type=T(w.neuron_type, torch.uint8),
                         vac_axon=T(w.vac_axon, torch.int32), sigma=w.sigma, seed=w.seed + k))
    b = msp.Batch(sims, graph=True, autotune=True)
    b.run(0.3, 0)
    b.run(0.3, 0)                       # the replay of the captured graph
    torch.cuda.synchronize()
    assert b.status() == [0] * len(ws)
    rng = np.random.default_rng(404)
    checked = small = 0
    for k, w in enumerate(ws):
        tgt, off = b.results(k)
        g = tgt.cpu().numpy().astype(np.int64)
        t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
        t.update_counts(w.vac_exc, w.vac_inh)
        ooff, src, elem = orc.search_list(w.vac_axon)
        assert np.array_equal(off.cpu().numpy(), ooff), k
        if w.n <= (1 << 14):
            q = np.arange(src.size)
            small += 1
        else:
            q = np.sort(rng.choice(src.size, size=min(20000, src.size), replace=False))
        o = t.find_targets(w.neuron_type, w.sigma, 0.3, w.seed + k, 0, src[q], elem[q])
        compare_targets(g[q], o, f"sim {k} n={w.n}")
        checked += q.size
        del t
    say(f"64 simulations: {small} checked in full, {checked} searches against the oracle")
    b.free()
    for d in sims:
        d["tree"].free()
