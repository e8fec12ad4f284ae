"""The electrical activity on the GPU (msp_activity_run) against the oracle: every state
array (v, u, calcium, frequencies as float64 bits; spikes, epoch counts, the last
step's inputs as integers) equal bitwise after runs that cross epoch boundaries, with
every spike exchanged, with the frequency approximation between ranks, and with it on
every synapse; at 65 536 neurons over 250 steps and at 8 388 608 neurons over the
steps around an epoch boundary."""
import numpy as np
import pytest
import torch

import paper_2509_26193_amd as msp
from oracle import oracle as orc
from gpu_util import T, say

pytestmark = pytest.mark.gpu


def _net(n, m, seed):
    rng = np.random.default_rng(seed)
    ty = (rng.random(n) < 0.2).astype(np.uint8)
    src = rng.integers(0, n, m).astype(np.int32)
    tgt = rng.integers(0, n, m).astype(np.int32)
    rank = (np.arange(n, dtype=np.int64) * 8 // n).astype(np.int32)
    return ty, src, tgt, ty[src].copy(), rank


def _pair(ty, seed=0, spk_share=0.0, freq_hi=0.0):
    """Device and oracle states, equal, optionally with preset spikes and frequencies."""
    o = orc.Activity(ty)
    if spk_share or freq_hi:
        rng = np.random.default_rng(seed)
        o.spk[:] = (rng.random(ty.size) < spk_share).astype(np.uint8)
        o.freq[:] = rng.random(ty.size) * freq_hi
    g = msp.Activity(T(ty, torch.uint8))
    for a, b in ((g.v, o.v), (g.u, o.u), (g.calcium, o.ca), (g.spiked, o.spk),
                 (g.count, o.count), (g.freq, o.freq)):
        a.copy_(torch.as_tensor(b))
    return g, o


def _same(g, o, li_g, li_o, label):
    torch.cuda.synchronize()
    for name, a, b in (("v", g.v, o.v), ("u", g.u, o.u), ("calcium", g.calcium, o.ca),
                       ("freq", g.freq, o.freq)):
        x = a.cpu().numpy()
        assert np.array_equal(x.view(np.uint64), b.view(np.uint64)), (label, name,
                                                                       np.abs(x - b).max())
    assert np.array_equal(g.spiked.cpu().numpy(), o.spk), label
    assert np.array_equal(g.count.cpu().numpy(), o.count), label
    assert np.array_equal(li_g.cpu().numpy(), li_o), label


@pytest.mark.parametrize("approx", [0, 1, 2])
def test_activity_matches_oracle_65536(approx):
    n, m = 65536, 200000
    ty, src, tgt, sty, rank = _net(n, m, seed=4)
    g, o = _pair(ty)
    spikes = torch.zeros(1, dtype=torch.int64, device="cuda")
    args = (T(src, torch.int32), T(tgt, torch.int32), T(sty, torch.uint8))
    li_g = g.run(*args, seed=11, t0=0, steps=250, approx=approx, rank=T(rank, torch.int32),
                 last_input=True, spikes=spikes)
    total, li_o = o.run(src, tgt, sty, seed=11, t0=0, steps=250, approx=approx, rank=rank,
                        last_input=True)
    say(f"[activity 65536 approx={approx}] {total} spikes in 250 steps "
        f"({total / n / 0.25:.1f} Hz)")
    assert int(spikes.item()) == total > 0
    _same(g, o, li_g, li_o, f"approx {approx}")


def test_activity_8388608_around_an_epoch_boundary():
    n, m = 1 << 23, 1 << 23
    ty, src, tgt, sty, rank = _net(n, m, seed=6)
    g, o = _pair(ty, seed=7, spk_share=0.05, freq_hi=0.05)
    spikes = torch.zeros(1, dtype=torch.int64, device="cuda")
    li_g = g.run(T(src, torch.int32), T(tgt, torch.int32), T(sty, torch.uint8), seed=12,
                 t0=95, steps=10, approx=1, rank=T(rank, torch.int32), last_input=True,
                 spikes=spikes)
    total, li_o = o.run(src, tgt, sty, seed=12, t0=95, steps=10, approx=1, rank=rank,
                        last_input=True)
    say(f"[activity 8M] {total} spikes in steps 95..104")
    assert int(spikes.item()) == total
    _same(g, o, li_g, li_o, "8M")


def test_activity_rejects_bad_synapses():
    ty, src, tgt, sty, rank = _net(1000, 100, seed=8)
    src[17] = 1000                                  # outside [0, n)
    g = msp.Activity(T(ty, torch.uint8))
    with pytest.raises(msp.MspError):
        g.run(T(src, torch.int32), T(tgt, torch.int32), T(sty, torch.uint8), seed=1, t0=0,
              steps=3)
    with pytest.raises(msp.MspError):                # approx 1 needs ranks
        g.run(T(src[:10], torch.int32), T(tgt[:10], torch.int32), T(sty[:10], torch.uint8),
              seed=1, t0=0, steps=1, approx=1)


@pytest.mark.parametrize("approx", [0, 1])
def test_activity_split_runs_equal_one_run(approx):
    """Runs continue from the state of the last one: the spikes recorded in a run's last
    step reach their targets in the first step of the next run."""
    n, m = 65536, 300000
    ty, src, tgt, sty, rank = _net(n, m, seed=9)
    g, o = _pair(ty, seed=10, spk_share=0.02, freq_hi=0.05)
    args = (T(src, torch.int32), T(tgt, torch.int32), T(sty, torch.uint8))
    g.run(*args, seed=13, t0=40, steps=70, approx=approx, rank=T(rank, torch.int32))
    li_g = g.run(*args, seed=13, t0=110, steps=50, approx=approx, rank=T(rank, torch.int32),
                 last_input=True)
    total, li_o = o.run(src, tgt, sty, seed=13, t0=40, steps=120, approx=approx, rank=rank,
                        last_input=True)
    say(f"[activity split runs approx={approx}] {total} spikes in 120 steps")
    _same(g, o, li_g, li_o, f"split approx {approx}")
