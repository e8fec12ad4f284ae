"""Writes attraction_262144_fd.txt: central differences of the oracle's frozen-set
forward L = sum_i log Z_i on the 262,144-neuron attraction workload (positions uniform
in a 5000 um cube, sigma = 750 um, theta = 0.3), with h = 1e-3 um, in 64 seeded
position coordinates and in sigma. Z_i is the level-0 normaliser of the Barnes-Hut
list of source i (Sec. III-B, "Division of work"); the accepted sets are held at the
unperturbed geometry. Calls only the oracle; run from the repository root:

    python tests/golden/make_attraction_fd.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from synth_inputs import config_attraction  # noqa: E402

H = 1e-3
N_COORDS = 64
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "attraction_262144_fd.txt")


def coordinates(n, k=N_COORDS, seed=2024):
    """k distinct (neuron, axis) pairs, seeded."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(3 * n, size=k, replace=False)
    return [(int(q // 3), int(q % 3)) for q in np.sort(idx)]


def main():
    w = config_attraction()
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    rows = []
    for k, (i, a) in enumerate(coordinates(w.n)):
        fd = t.frozen_derivative(w.neuron_type, w.vac_axon, w.sigma, w.theta, H, coord=(i, a))
        rows.append(f"{i} {a} {fd:.17e}")
        print(f"{k + 1}/{N_COORDS}: x[{i},{a}] {fd:.10e}", flush=True)
    fd_s = t.frozen_derivative(w.neuron_type, w.vac_axon, w.sigma, w.theta, H)
    rows.append(f"sigma - {fd_s:.17e}")
    with open(OUT, "w") as f:
        f.write("# Central differences (h = 1e-3 um) of the fp64 oracle's frozen-set forward\n"
                "# L = sum_i log Z_i, Z_i = level-0 Barnes-Hut normaliser of source i\n"
                "# (Sec. III-B, Division of work), on the 262,144-neuron attraction workload\n"
                "# (uniform in a 5000 um cube, sigma 750 um, theta 0.3; synth_inputs.\n"
                "# config_attraction). Written by tests/golden/make_attraction_fd.py.\n"
                "# neuron axis dL/dx   (last line: sigma - dL/dsigma)\n")
        f.write("\n".join(rows) + "\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
