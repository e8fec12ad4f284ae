"""The stored central differences of the 262,144-neuron attraction workload
(tests/golden/attraction_262144_fd.txt, written by make_attraction_fd.py from the
oracle alone) are what the oracle gives now: one coordinate and sigma recomputed."""
import os
import sys

import numpy as np

from oracle import oracle as orc
from synth_inputs import config_attraction

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_attraction_fd as mk  # noqa: E402


def test_golden_central_differences_reproduce():
    rows = {}
    with open(mk.OUT) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            a, b, v = ln.split()
            rows[(a, b)] = float(v)
    w = config_attraction()
    coords = mk.coordinates(w.n)
    assert len(rows) == len(coords) + 1
    assert all((str(i), str(a)) in rows for i, a in coords)
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    i, a = coords[0]
    fd = t.frozen_derivative(w.neuron_type, w.vac_axon, w.sigma, w.theta, mk.H, coord=(i, a))
    assert np.isclose(fd, rows[(str(i), str(a))], rtol=1e-12, atol=0.0)
    fd_s = t.frozen_derivative(w.neuron_type, w.vac_axon, w.sigma, w.theta, mk.H)
    assert np.isclose(fd_s, rows[("sigma", "-")], rtol=1e-12, atol=0.0)
