"""Pins of the oracle's plasticity step (the change of the network between two
connectivity updates, Sec. III-A) against closed forms, distributions and invariants:

* the growth rule is zero at the growth onset and at the target calcium, largest
  (steps * nu) midway, symmetric about it, and tends to -steps * nu far away;
* the calcium draw is N(mean, sd) (Kolmogorov-Smirnov over many draws, independent
  between element kinds);
* a step deletes exactly round(frac * m) synapses when no element retracts, each with
  probability frac over many steps;
* where floor(z) falls below the bound elements, exactly that many of the neuron's
  synapses break, each equally likely over many steps;
* bound elements always equal the synapse counts, vacancies are floor(z) - bound >= 0.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as orc


def test_growth_rule_closed_form():
    nu, eps, eta, steps = 0.001, 0.7, 0.4, 100
    xi = 0.5 * (eps + eta)
    assert abs(orc.growth_delta(eps)) < 1e-15
    assert abs(orc.growth_delta(eta)) < 1e-15
    assert orc.growth_delta(xi) == pytest.approx(steps * nu, rel=1e-15)
    for d in (0.01, 0.07, 0.2):
        assert orc.growth_delta(xi - d) == pytest.approx(orc.growth_delta(xi + d), rel=1e-12)
    assert orc.growth_delta(-5.0) == pytest.approx(-steps * nu, rel=1e-12)
    assert orc.growth_delta(0.3) < 0.0 < orc.growth_delta(0.5)
    # 2 exp(-r^2) - 1 = 0 at r = sqrt(ln 2): the onset and the target lie that far
    # from the midpoint in units of zeta
    zeta = (eps - eta) / (2.0 * math.sqrt(math.log(2.0)))
    assert (eps - xi) / zeta == pytest.approx(math.sqrt(math.log(2.0)), rel=1e-15)


def test_calcium_is_normal_and_independent():
    draws = np.array([orc.calcium(42, j, 0, 3) for j in range(40000)])
    assert draws.mean() == pytest.approx(0.7, abs=3e-3)
    assert draws.std() == pytest.approx(0.1, rel=2e-2)
    assert stats.kstest((draws - 0.7) / 0.1, "norm").pvalue > 1e-3
    other = np.array([orc.calcium(42, j, 1, 3) for j in range(40000)])
    assert abs(np.corrcoef(draws, other)[0, 1]) < 0.03
    assert orc.calcium(42, 5, 2, 7) == orc.calcium(42, 5, 2, 7)
    assert orc.calcium(42, 5, 2, 7) != orc.calcium(43, 5, 2, 7)


def _network(n=400, m=3000, seed=0, z0=3.0):
    rng = np.random.default_rng(seed)
    net = orc.Network(np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int32),
                      capacity=m)
    net.z[:] = z0 + 0.5                      # room for the synapses recorded below
    src = rng.integers(0, n, m).astype(np.int32)
    tgt = rng.integers(0, n, m).astype(np.int32)
    ty = rng.integers(0, 2, m).astype(np.uint8)
    # keep the bound elements within z: at most 3 synapses per element kind and neuron
    keep = np.ones(m, bool)
    cnt = np.zeros((3, n), np.int64)
    for s in range(m):
        a, b = src[s], 1 + int(ty[s])
        if cnt[0, a] >= z0 or cnt[b, tgt[s]] >= z0:
            keep[s] = False
            continue
        cnt[0, a] += 1
        cnt[b, tgt[s]] += 1
    net.record(src[keep], tgt[keep], ty[keep])
    return net


def _check_books(net):
    src, tgt, ty = net.synapses()
    n = net.n
    assert np.array_equal(net.bound[0], np.bincount(src, minlength=n))
    assert np.array_equal(net.bound[1], np.bincount(tgt[ty == 0], minlength=n))
    assert np.array_equal(net.bound[2], np.bincount(tgt[ty == 1], minlength=n))


def test_deletion_count_and_uniformity():
    grow = dict(ca_mean=0.55, ca_sd=1e-9)     # z grows: nothing retracts
    base = _network()
    m0 = base.m
    hits = np.zeros(m0)
    trials = 400
    for step in range(trials):
        net = _network()
        before = net.synapses()
        vac = net.step(11, step, grow)
        _check_books(net)
        assert net.m == m0 - int(math.floor(0.1 * m0 + 0.5))
        assert all(np.all(v >= 0) for v in vac)
        # which synapses went (the list keeps its order)
        key_before = before[0].astype(np.int64) * 1_000_000 + before[1] * 2 + before[2]
        src, tgt, ty = net.synapses()
        key_after = src.astype(np.int64) * 1_000_000 + tgt * 2 + ty
        gone = np.ones(m0, bool)
        j = 0
        for s in range(m0):               # subsequence match (order is kept)
            if j < key_after.size and key_before[s] == key_after[j]:
                gone[s] = False
                j += 1
        assert j == key_after.size
        hits += gone
    freq = hits / trials
    assert freq.mean() == pytest.approx(0.1, rel=1e-3)
    # each synapse deleted with probability 0.1: binomial spread of the counts
    chi2 = ((hits - 0.1 * trials) ** 2 / (0.1 * trials * 0.9)).sum()
    assert stats.chi2.sf(chi2, m0 - 1) > 1e-4


def test_retraction_breaks_exactly_the_excess_uniformly():
    n = 50
    counts = np.zeros(6)
    trials = 3000
    for step in range(trials):
        net = orc.Network(np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int32),
                          capacity=16)
        net.z[:] = 10.0
        # neuron 0 sends 6 synapses; its axonal z sits just above 6 and will drop below
        net.record(np.zeros(6, np.int32), np.arange(1, 7, dtype=np.int32),
                   np.zeros(6, np.uint8))
        net.z[0, 0] = 6.02
        vac = net.step(5, step, dict(ca_mean=-5.0, ca_sd=1e-9, delete_frac=0.0))
        _check_books(net)
        # z fell by ~0.1 to ~5.92: exactly one of the six synapses broke
        assert net.z[0, 0] == pytest.approx(6.02 - 0.1, abs=1e-9)
        assert net.m == 5 and net.bound[0, 0] == 5 and vac[0][0] == 0
        src, tgt, _ = net.synapses()
        broken = sorted(set(range(1, 7)) - set(tgt.tolist()))
        assert len(broken) == 1
        counts[broken[0] - 1] += 1
        # every z fell from 10 to ~9.9: the freed dendritic element of the broken
        # synapse's target is vacant again, the other targets still bind one
        assert vac[1][broken[0]] == 9
        assert all(vac[1][g] == 8 for g in range(1, 7) if g != broken[0])
    assert stats.chisquare(counts).pvalue > 1e-4


def test_bookkeeping_over_many_steps():
    net = _network(n=300, m=2000, seed=4)
    for step in range(20):
        vac = net.step(9, step)
        _check_books(net)
        assert np.all(net.bound <= np.floor(net.z))
        for k in range(3):
            assert np.array_equal(vac[k], (np.floor(net.z[k]) - net.bound[k]).astype(np.int32))
        assert np.all(net.z >= 0.0)
