"""The working memory the library keeps per device is shared by searches, commits and
plasticity steps: one call holds it at a time, and a call's stream waits for the kernels
of the previous user before they are overwritten. Two simulations updated alternately on
two streams (each call on its own stream, no host wait between them beyond the calls'
own status reads) must give exactly what the same calls give one after the other on one
stream, also across a release of that memory."""
import numpy as np
import pytest
import torch

import paper_2509_26193_amd as msp
from synth_inputs import uniform_cube
from gpu_util import T, say

pytestmark = pytest.mark.gpu


def _sim(n, seed):
    edge = 20000.0 * (n / float(1 << 23)) ** (1.0 / 3.0)    # the 8M workload's density
    w = uniform_cube(n, edge, seed=seed)
    return w


def _state(w):
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    vac = [T(v, torch.int32) for v in (w.vac_axon, w.vac_exc, w.vac_inh)]
    return dict(w=w, tree=tree, ty=T(w.neuron_type, torch.uint8), vac=vac)


def _find(s, step):
    w = s["w"]
    msp.update_vacant_counts(s["tree"], s["vac"][1], s["vac"][2])
    s["tgt"], s["off"] = msp.find_targets(s["tree"], s["ty"], s["vac"][0], w.sigma, w.theta,
                                          w.seed, step)


def _commit(s, step):
    w = s["w"]
    va, ve, vi = s["vac"]
    r = msp.commit_synapses(s["tgt"], s["off"], s["ty"], va, ve, vi, w.seed, step)
    s["res"] = (s["tgt"], r["syn_src"], r["syn_tgt"], r["syn_type"], va, ve, vi)


def _run(streams, release_at=None):
    sims = [_state(_sim(65536, 21)), _state(_sim(40000, 22))]
    torch.cuda.synchronize()                         # built on the current stream
    outs = []
    for step in range(3):
        if step == release_at:
            torch.cuda.synchronize()
            msp.release_workspace()
        for k, s in enumerate(sims):                 # both searches, then both commits
            with torch.cuda.stream(streams[k]):
                _find(s, step)
        for k, s in enumerate(sims):
            with torch.cuda.stream(streams[k]):
                _commit(s, step)
        torch.cuda.synchronize()
        outs.append([[x.cpu().numpy().copy() for x in s["res"]] for s in sims])
    for s in sims:
        s["tree"].free()
    torch.cuda.synchronize()
    return outs


def test_two_streams_share_the_kept_working_memory():
    one = torch.cuda.current_stream()
    ref = _run([one, one])
    two = [torch.cuda.Stream(), torch.cuda.Stream()]
    got = _run(two)
    rel = _run(two, release_at=1)
    for step in range(3):
        for k in range(2):
            for a, b, c in zip(ref[step][k], got[step][k], rel[step][k]):
                assert np.array_equal(a, b) and np.array_equal(a, c), (step, k)
        say(f"update {step}: both simulations equal on two streams and after a release")
