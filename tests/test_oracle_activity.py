"""Pins of the oracle's electrical activity (Sec. II, "Update of electrical activity")
and of its firing-rate approximation (Sec. IV-B), each against something other than the
oracle's own formulas: brute-force spike routing, the closed-form resting state of the
Izhikevich neuron, the closed form of the calcium average, exact epoch frequencies,
the binomial statistics of the frequency draws, and bitwise resumption."""
import math

import numpy as np

from oracle import oracle as orc


def _net(n=3000, m=9000, seed=1):
    rng = np.random.default_rng(seed)
    ty = (rng.random(n) < 0.2).astype(np.uint8)
    src = rng.integers(0, n, m).astype(np.int32)
    tgt = rng.integers(0, n, m).astype(np.int32)
    return ty, src, tgt, ty[src].copy()


def test_spikes_reach_their_targets():
    ty, src, tgt, sty = _net()
    a = orc.Activity(ty)
    rng = np.random.default_rng(2)
    a.spk[:] = (rng.random(ty.size) < 0.3).astype(np.uint8)
    sent = a.spk.copy()
    _, li = a.run(src, tgt, sty, seed=7, t0=3, steps=1, last_input=True)
    hit = sent[src] != 0
    assert np.array_equal(li[0], np.bincount(tgt[hit & (sty == 0)], minlength=ty.size))
    assert np.array_equal(li[1], np.bincount(tgt[hit & (sty == 1)], minlength=ty.size))


def test_rank_split_of_the_approximation():
    ty, src, tgt, sty = _net(seed=3)
    rank = (np.arange(ty.size) * 4 // ty.size).astype(np.int32)
    local = rank[src] == rank[tgt]
    # every neuron spiked, no frequency yet: only local synapses carry a spike
    a = orc.Activity(ty)
    a.spk[:] = 1
    _, li = a.run(src, tgt, sty, seed=7, t0=3, steps=1, approx=1, rank=rank, last_input=True)
    assert np.array_equal(li.sum(0), np.bincount(tgt[local], minlength=ty.size))
    # nobody spiked, frequency 1: only the synapses between ranks carry one
    a = orc.Activity(ty)
    a.freq[:] = 1.0
    _, li = a.run(src, tgt, sty, seed=7, t0=3, steps=1, approx=1, rank=rank, last_input=True)
    assert np.array_equal(li.sum(0), np.bincount(tgt[~local], minlength=ty.size))


def test_frequency_draws_are_bernoulli():
    # one synapse per target, so each synapse's arrival is visible
    m = 200000
    ty = np.zeros(m, np.uint8)
    src = np.arange(m, dtype=np.int32)
    tgt = np.roll(src, 1)
    f = 0.25
    got = []
    for t in (10, 11):
        a = orc.Activity(ty)
        a.freq[:] = f
        _, li = a.run(src, tgt, ty[src], seed=9, t0=t, steps=1, approx=2, last_input=True)
        got.append(li[0][tgt] > 0)
    sd = math.sqrt(m * f * (1 - f))
    for g in got:
        assert abs(int(g.sum()) - m * f) < 5 * sd
    both = int((got[0] & got[1]).sum())          # independent across steps
    assert abs(both - m * f * f) < 5 * math.sqrt(m * f * f * (1 - f * f))


def test_resting_state_below_rheobase():
    # constant input I below the saddle-node point: no spike, and v, u settle on the
    # stable root of 0.04 v^2 + (5 - b) v + 140 + I = 0, u = b v
    for ty_ in (0, 1):
        a = orc.Activity(np.array([ty_], np.uint8), dict(bg_mean=3.0, bg_width=0.0))
        assert a.run(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint8),
                     seed=1, t0=0, steps=4000) == 0
        b = a.p["b_inh"] if ty_ else a.p["b_exc"]
        disc = (5.0 - b) ** 2 - 4 * 0.04 * (140.0 + 3.0)
        vstar = (-(5.0 - b) - math.sqrt(disc)) / (2 * 0.04)
        assert abs(a.v[0] - vstar) < 1e-9
        assert abs(a.u[0] - b * vstar) < 1e-9


def _trace(I, steps, ty_=0, params=None):
    p = dict(bg_mean=I, bg_width=0.0, **(params or {}))
    a = orc.Activity(np.array([ty_], np.uint8), p)
    none_i, none_u = np.zeros(0, np.int32), np.zeros(0, np.uint8)
    spk, v, ca, freq = [], [], [], []
    for t in range(steps):
        a.run(none_i, none_i, none_u, seed=1, t0=t, steps=1)
        spk.append(int(a.spk[0]))
        v.append(a.v[0])
        ca.append(a.ca[0])
        freq.append(a.freq[0])
    return a, np.array(spk), np.array(v), np.array(ca), np.array(freq)


def test_tonic_spiking_resets():
    # constant input above the saddle-node point: the neuron keeps firing, and every
    # spike leaves v exactly at c (the overshoot of the 1 ms step feeds u, so the
    # intervals vary between 40 and 70 steps instead of repeating exactly)
    for ty_, c in ((0, "c_exc"), (1, "c_inh")):
        a, spk, v, _, _ = _trace(10.0, 1000, ty_)
        t = np.nonzero(spk)[0]
        assert t.size > 10
        assert np.all(v[t] == a.p[c])
        assert np.diff(t).max() < 100


def test_calcium_is_the_decaying_sum_of_spikes():
    a, spk, _, ca, _ = _trace(10.0, 1500)
    r = 1.0 - 1.0 / a.p["ca_tau"]
    T = spk.size - 1
    expect = sum(a.p["ca_beta"] * r ** (T - k) for k in np.nonzero(spk)[0])
    assert abs(ca[-1] - expect) <= 1e-12 * max(1.0, expect)


def test_epoch_frequency_is_spikes_per_step():
    a, spk, _, _, freq = _trace(10.0, 300)
    for e in range(3):
        assert freq[100 * e + 99] == spk[100 * e:100 * e + 100].sum() / 100.0
    assert freq[150] == freq[99]                      # held through the next epoch


def test_resume_is_bitwise():
    ty, src, tgt, sty = _net(seed=5)
    full = orc.Activity(ty)
    n_full = full.run(src, tgt, sty, seed=3, t0=0, steps=240, approx=2)
    half = orc.Activity(ty)
    n1 = half.run(src, tgt, sty, seed=3, t0=0, steps=130, approx=2)
    n2 = half.run(src, tgt, sty, seed=3, t0=130, steps=110, approx=2)
    assert n_full == n1 + n2 > 0
    for k in ("v", "u", "ca", "spk", "count", "freq"):
        assert np.array_equal(getattr(full, k), getattr(half, k)), k
