"""The search sweep drops its own-cell test (an inner node holding the source's leaf is
always opened) when theta <= 1/2 and every position lies inside the cube: the source
and the node's centroid then share a cell of edge l, so d^2 <= 3 l^2 and the
acceptance test l^2 < theta^2 d^2 cannot pass. Checked here on the oracle's trees and
centroids, at theta = 1/2: never passes for positions inside the cube (uniform,
clustered, coincident), and does pass for positions outside it, where the test is kept."""
import numpy as np
import pytest

from oracle import oracle as orc


def _own_cell_acceptances(pos, theta, box_min=(0.0, 0.0, 0.0), edge=1000.0):
    n = pos.shape[0]
    t = orc.OracleTree(pos, np.asarray(box_min, dtype=np.float64), edge)
    ones = np.ones(n, np.int32)
    t.update_counts(ones, ones)
    nd = t.nodes()
    cnt, cen = t.aggregates(0)
    order, _ = t.order()
    se, dep, beg, end = nd["subtree_end"], nd["depth"], nd["begin"], nd["end"]
    N = dep.size
    leaf = np.empty(n, np.int64)
    inner = np.zeros(N, bool)
    for x in range(N):
        if se[x] > x + 1:
            inner[x] = True
        else:
            leaf[order[beg[x]:end[x]]] = x
    hits = 0
    for x in np.nonzero(inner & (cnt > 0))[0]:
        mine = (leaf >= x) & (leaf < se[x])
        d2 = ((pos[mine] - cen[x]) ** 2).sum(axis=1)
        hits += int(np.sum(edge * edge < np.ldexp(theta * theta * d2, 2 * int(dep[x]))))
    return hits


@pytest.mark.parametrize("kind", ["uniform", "clusters", "coincident", "corners"])
def test_own_cell_never_accepted_inside_the_cube(kind):
    rng = np.random.default_rng(3)
    if kind == "uniform":
        pos = rng.uniform(0, 1000, size=(3000, 3))
    elif kind == "clusters":
        c = rng.uniform(100, 900, size=(6, 3))
        pos = np.clip(np.repeat(c, 400, axis=0) + rng.normal(0, 20, size=(2400, 3)), 0, 1000)
    elif kind == "coincident":
        pos = np.repeat(rng.uniform(0, 1000, size=(50, 3)), 8, axis=0)
    else:   # on the faces and corners of the cube, where cells are clamped
        pos = rng.integers(0, 2, size=(500, 3)) * 1000.0 + rng.uniform(-1e-9, 0, size=(500, 3))
        pos = np.clip(pos, 0, 1000)
    assert _own_cell_acceptances(pos, 0.5) == 0


def test_own_cell_accepted_outside_the_cube():
    rng = np.random.default_rng(11)
    pos = rng.uniform(-400, 1400, size=(300, 3))
    assert _own_cell_acceptances(pos, 0.3) > 0
