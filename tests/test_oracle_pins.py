"""Pins of the fp64 CPU oracle against things other than itself.

* Philox4x64-10 against numpy.random.Philox and the published known-answer vector.
* Morton keys against their closed form (bit interleave, decode round trip).
* The octree and its aggregates against an independent insertion-built octree.
* theta = 0 search against the O(n) direct solution (the paper, Sec. II: theta = 0
  yields the direct solution), bitwise.
* theta > 0 search against an independent Python Barnes-Hut, and the empirical
  target frequencies against the exact implied distribution (chi-square).
* Special cases: one neuron, two neurons, all vacancy on one neuron.
* Commit against a brute-force sort, its invariants, and the acceptance law v/r.
* The expected-attraction adjoint against a closed form, central differences and a
  direct theta = 0 gradient.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as orc
from synth_inputs import uniform_cube, config_small
import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- Philox
def test_philox_matches_numpy():
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        ctr[0] |= 1  # nonzero so that numpy's pre-decrement never wraps below zero here
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        _, r = brute.philox_u(key[0], key[1], tuple(ctr))
        out = orc.philox4x64_10(ctr, key)
        assert int(out[0]) == r


def test_philox_known_answer():
    # tests/golden/philox4x64_10_kat.txt: counter, key, expected block
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert rows
    for r in rows:
        vals = [int(x, 16) for x in r]
        ctr, key, want = vals[0:4], vals[4:6], vals[6:10]
        got = orc.philox4x64_10(ctr, key)
        assert [int(x) for x in got] == want


# --------------------------------------------------------------------------- keys
def _interleave(q):
    qx, qy, qz = q
    k = 0
    for b in range(20, -1, -1):
        k = (k << 3) | (((qx >> b) & 1) << 2) | (((qy >> b) & 1) << 1) | ((qz >> b) & 1)
    return k


def _deinterleave(k):
    q = [0, 0, 0]
    for b in range(21):
        d = (k >> (3 * b)) & 7
        q[0] |= ((d >> 2) & 1) << b
        q[1] |= ((d >> 1) & 1) << b
        q[2] |= (d & 1) << b
    return tuple(q)


def test_keys_closed_form_and_order():
    w = uniform_cube(500, 1000.0, seed=3)
    pos = w.pos.copy()
    pos[7] = pos[3]          # duplicate point
    pos[11] = [-5.0, 1000.0, 2000.0]   # outside the cube: clamped
    t = orc.OracleTree(pos, np.zeros(3), 1000.0)
    order, keys = t.order()
    for i in range(pos.shape[0]):
        q = tuple(brute.quantise(pos[i, a], 0.0, 1000.0) for a in range(3))
        assert int(keys[i]) == _interleave(q)
        assert _deinterleave(int(keys[i])) == q
    assert brute.quantise(-5.0, 0.0, 1000.0) == 0
    assert brute.quantise(2000.0, 0.0, 1000.0) == 2**21 - 1
    ref = np.lexsort((np.arange(pos.shape[0]), keys))
    assert np.array_equal(order, ref)


# --------------------------------------------------------------------------- tree
def _tree_cases():
    rng = np.random.default_rng(11)
    cases = []
    for n in (1, 2, 3, 9, 40, 150):
        cases.append(rng.uniform(0, 1000, size=(n, 3)))
    p = rng.uniform(0, 1000, size=(30, 3))
    p[5] = p[6] = p[7] = p[2]                      # coincident: a depth-21 bucket
    p[10] = p[9] + 1e-6                            # same quantised cell, distinct ids
    cases.append(p)
    p = np.full((12, 3), 500.0)                    # all coincident
    cases.append(p)
    c = rng.uniform(0, 1000, size=(3, 3))
    cases.append(np.repeat(c, 20, axis=0) + rng.normal(0, 0.01, size=(60, 3)))  # chains
    return cases


@pytest.mark.parametrize("case", range(9))
def test_tree_and_aggregates_match_insertion_tree(case):
    pos = _tree_cases()[case]
    n = pos.shape[0]
    rng = np.random.default_rng(100 + case)
    ve = rng.integers(0, 4, size=n).astype(np.int32)
    vi = rng.integers(0, 4, size=n).astype(np.int32)
    t = orc.OracleTree(pos, np.zeros(3), 1000.0)
    t.update_counts(ve, vi)
    ref = brute.InsertTree(pos, (0.0, 0.0, 0.0), 1000.0)
    cells = ref.preorder()
    nodes = t.nodes()
    order, _ = t.order()
    assert t.num_nodes == len(cells)
    for k, c in enumerate(cells):
        assert nodes["depth"][k] == c.depth
        assert bool(nodes["is_leaf"][k]) == c.leaf
        members = sorted(int(x) for x in order[nodes["begin"][k]:nodes["end"][k]])
        assert members == sorted(ref.leaves_in_order(c))
    for ty, vac in ((0, ve), (1, vi)):
        agg = ref.aggregate([int(x) for x in vac])
        v, cen = t.aggregates(ty)
        for k, c in enumerate(cells):
            rv, rc = agg[id(c)]
            assert v[k] == rv
            if rv > 0:
                assert tuple(float(x) for x in cen[k]) == rc   # bitwise


def test_tree_invariants_4096():
    w = config_small()
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    nd = t.nodes()
    N = t.num_nodes
    order, keys = t.order()
    leaf = nd["is_leaf"].astype(bool)
    # every neuron in exactly one leaf
    cover = np.zeros(w.n, np.int64)
    for k in np.nonzero(leaf)[0]:
        cover[order[nd["begin"][k]:nd["end"][k]]] += 1
    assert np.all(cover == 1)
    # inner nodes hold >= 2 neurons; leaves hold one unless at depth 21
    size = nd["end"] - nd["begin"]
    assert np.all(size[~leaf] >= 2)
    assert np.all((size[leaf] == 1) | (nd["depth"][leaf] == 21))
    # pre-order subtree intervals: a leaf is its own subtree
    assert np.all(nd["subtree_end"][leaf] == np.nonzero(leaf)[0] + 1)
    assert nd["subtree_end"][0] == N
    for ty, vac in ((0, w.vac_exc), (1, w.vac_inh)):
        v, cen = t.aggregates(ty)
        assert v[0] == int(vac.sum())
        # v of an inner node = sum over the leaves below
        for k in range(0, N, 37):
            ids = order[nd["begin"][k]:nd["end"][k]]
            assert v[k] == int(vac[ids].sum())
            if v[k] > 0:
                # centroid inside the cell box (up to rounding)
                l = w.box_edge / 2 ** nd["depth"][k]
                lo = np.floor((w.pos[ids].min(0) - w.box_min) / l) * l + w.box_min
                assert np.all(cen[k] >= lo - 1e-9 * w.box_edge)
                assert np.all(cen[k] <= lo + l + 1e-9 * w.box_edge)


# --------------------------------------------------------------------------- search
def _all(t, w, sigma, theta, seed=42, step=0):
    off, src, elem = orc.search_list(w.vac_axon)
    r = t.find_targets(w.neuron_type, sigma, theta, seed, step, src, elem)
    return off, src, elem, r


def test_theta0_equals_direct_solution():
    w = uniform_cube(96, 1000.0, seed=5)
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    order, _ = t.order()
    off, src, elem, r = _all(t, w, 750.0, 0.0)
    assert src.size > 50
    for q in range(src.size):
        i, j = int(src[q]), int(elem[q])
        vac = w.vac_inh if w.neuron_type[i] else w.vac_exc
        g, Z = brute.brute_theta0(w.pos, order, vac, i, j, 750.0, 42, 0)
        assert r["target"][q] == g
        assert r["z0"][q] == Z            # bitwise: same terms, same order
        assert r["levels"][q] == 1        # theta = 0 never accepts a cell


def test_theta_tiny_equals_theta0():
    w = uniform_cube(80, 1000.0, seed=8)
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    a = _all(t, w, 750.0, 0.0)[3]
    b = _all(t, w, 750.0, 1e-9)[3]
    assert np.array_equal(a["target"], b["target"])
    assert np.array_equal(a["z0"], b["z0"])


@pytest.mark.parametrize("theta", [0.2, 0.3, 0.5, 0.9])
def test_search_matches_independent_python_bh(theta):
    w = uniform_cube(120, 1000.0, seed=21)
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    ref = brute.InsertTree(w.pos, (0.0, 0.0, 0.0), 1000.0)
    aggs = [ref.aggregate([int(x) for x in w.vac_exc]), ref.aggregate([int(x) for x in w.vac_inh])]
    vacs = [[int(x) for x in w.vac_exc], [int(x) for x in w.vac_inh]]
    off, src, elem, r = _all(t, w, 300.0, theta, seed=9, step=4)
    for q in range(src.size):
        i, j = int(src[q]), int(elem[q])
        ty = int(w.neuron_type[i])
        g, z0 = ref.search(aggs[ty], vacs[ty], i, j, 300.0, theta, 9, 4)
        assert r["target"][q] == g
        assert r["z0"][q] == z0
    # sanity: theta > 0 does accept cells somewhere
    assert theta < 0.3 or r["levels"].max() > 1


def _counted_cases():
    """(label, positions, cube edge) for the per-search output pins: the 120-neuron
    cube of the theta sweep and the degenerate trees."""
    rng = np.random.default_rng(21)
    cases = [("uniform120", uniform_cube(120, 1000.0, seed=21).pos)]
    for k, pos in enumerate(_tree_cases()):
        if pos.shape[0] >= 2:
            cases.append((f"tree{k}", pos))
    cases.append(("outside", rng.uniform(-300, 1300, size=(80, 3))))
    return cases


@pytest.mark.parametrize("theta", [0.0, 0.2, 0.3, 0.5, 0.9])
def test_window_and_work_counters_match_independent_search(theta):
    """The oracle's boundary distance of the draw (the only quantity that excuses a
    differing choice) and its visit/open/entry counters (the numerator of the roofline)
    per search, against an independent Barnes-Hut written from Sec. III-B ("Division of
    work": the list, the draw by probability, the restart): bitwise equal, and the
    distance equal to exact rational arithmetic on the same weights to 1e-12."""
    for label, pos in _counted_cases():
        n = pos.shape[0]
        rng = np.random.default_rng(7 + n)
        ve = rng.integers(0, 4, size=n).astype(np.int32)
        vi = rng.integers(0, 4, size=n).astype(np.int32)
        va = rng.integers(0, 3, size=n).astype(np.int32)
        ty = (rng.random(n) < 0.3).astype(np.uint8)
        t = orc.OracleTree(pos, np.zeros(3), 1000.0)
        t.update_counts(ve, vi)
        off, src, elem = orc.search_list(va)
        sigma = 300.0
        r = t.find_targets(ty, sigma, theta, 9, 4, src, elem)
        ref = brute.InsertTree(pos, (0.0, 0.0, 0.0), 1000.0)
        vacs = [[int(x) for x in ve], [int(x) for x in vi]]
        aggs = [ref.aggregate(vacs[0]), ref.aggregate(vacs[1])]
        restarts = 0
        for q in range(src.size):
            i, j = int(src[q]), int(elem[q])
            k = int(ty[i])
            b, exact = ref.search_full(aggs[k], vacs[k], i, j, sigma, theta, 9, 4)
            assert r["target"][q] == b["target"], (label, q)
            assert r["levels"][q] == b["levels"], (label, q)
            assert r["visits"][q] == b["visits"], (label, q, r["visits"][q], b["visits"])
            assert r["opens"][q] == b["opens"], (label, q, r["opens"][q], b["opens"])
            assert r["window"][q] == b["window"], (label, q, r["window"][q], b["window"])
            assert r["entries0"][q] == b["entries0"], (label, q)
            # the chosen entry's exact interval holds u, and the float distance is the
            # exact one up to the rounding of the running sums
            we = 1.0
            for u, lo, hi in exact:
                assert lo - 1e-12 <= u <= hi + 1e-12, (label, q)
                we = min(we, float(min(u - lo, hi - u)))
            assert abs(r["window"][q] - we) <= 1e-12, (label, q)
            restarts += max(0, b["levels"] - 1)
        if theta >= 0.3 and label == "uniform120":
            assert restarts > 0            # restart levels are exercised


def test_targets_valid_and_never_self():
    w = uniform_cube(2000, 1000.0, seed=4)
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    off, src, elem, r = _all(t, w, 200.0, 0.4)
    g = r["target"]
    assert np.all(g != src)
    ok = g >= 0
    vac = np.where(w.neuron_type[src[ok]] == 1, w.vac_inh[g[ok]], w.vac_exc[g[ok]])
    assert np.all(vac > 0)
    assert np.all(r["levels"] <= 22)


def test_implied_distribution_chi_square():
    from scipy import stats
    rng = np.random.default_rng(2)
    n = 60
    pos = rng.uniform(0, 1000, size=(n, 3))
    ve = rng.integers(0, 4, size=n).astype(np.int32)
    vi = rng.integers(0, 4, size=n).astype(np.int32)
    types = np.zeros(n, np.uint8)
    sigma, theta = 400.0, 0.6
    t = orc.OracleTree(pos, np.zeros(3), 1000.0)
    t.update_counts(ve, vi)
    ref = brute.InsertTree(pos, (0.0, 0.0, 0.0), 1000.0)
    vac = [int(x) for x in ve]
    agg = ref.aggregate(vac)
    for i in (0, 17):
        dist = ref.implied_distribution(agg, vac, i, sigma, theta)
        assert abs(sum(dist.values()) - 1.0) < 1e-12
        assert i not in dist
        M = 100_000
        r = t.find_targets(types, sigma, theta, 5, 0, np.full(M, i), np.arange(M))
        assert r["levels"].max() > 1          # restarts are exercised
        ids = sorted(dist)
        exp_ = np.array([dist[g] for g in ids]) * M
        obs = np.array([(r["target"] == g).sum() for g in ids], dtype=float)
        assert obs.sum() == M
        # merge bins with small expectation
        big = exp_ >= 5
        e2 = np.append(exp_[big], exp_[~big].sum())
        o2 = np.append(obs[big], obs[~big].sum())
        if e2[-1] == 0:
            e2, o2 = e2[:-1], o2[:-1]
        p = stats.chisquare(o2, e2).pvalue
        assert p > 1e-4, p


def test_special_cases():
    one = orc.OracleTree(np.array([[1.0, 2.0, 3.0]]), np.zeros(3), 10.0)
    one.update_counts(np.array([3], np.int32), np.array([3], np.int32))
    r = one.find_targets(np.zeros(1, np.uint8), 5.0, 0.3, 1, 0, [0, 0], [0, 1])
    assert list(r["target"]) == [-1, -1]

    two = np.array([[1.0, 1.0, 1.0], [8.0, 8.0, 8.0]])
    t = orc.OracleTree(two, np.zeros(3), 10.0)
    t.update_counts(np.array([2, 1], np.int32), np.array([0, 0], np.int32))
    ty = np.zeros(2, np.uint8)
    r = t.find_targets(ty, 5.0, 0.3, 1, 0, [0, 0, 1], [0, 1, 0])
    assert list(r["target"]) == [1, 1, 0]
    r = t.find_targets(np.ones(2, np.uint8), 5.0, 0.3, 1, 0, [0, 1], [0, 0])
    assert list(r["target"]) == [-1, -1]        # no inhibitory vacancy anywhere

    w = uniform_cube(500, 1000.0, seed=12)
    ve = np.zeros(500, np.int32)
    ve[123] = 5
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(ve, np.zeros(500, np.int32))
    src = np.array([i for i in range(500) if i != 123])
    r = t.find_targets(np.zeros(500, np.uint8), 750.0, 0.3, 3, 0, src, np.zeros_like(src))
    assert np.all(r["target"] == 123)
    r = t.find_targets(np.zeros(500, np.uint8), 750.0, 0.3, 3, 0, [123], [0])
    assert r["target"][0] == -1


def test_visits_grow_logarithmically():
    """O(n log n) overall (Sec. II): at fixed density each 8x step in n adds about one
    tree level, i.e. a roughly constant number of visits per search."""
    per = []
    for n in (4096, 32768, 262144):
        edge = 1000.0 * (n / 4096.0) ** (1.0 / 3.0)
        w = uniform_cube(n, edge, seed=1)
        t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
        t.update_counts(w.vac_exc, w.vac_inh)
        src = np.arange(0, n, max(1, n // 300))
        r = t.find_targets(w.neuron_type, 150.0, 0.3, 1, 0, src, np.zeros_like(src))
        per.append(r["visits"].mean())
    inc1, inc2 = per[1] - per[0], per[2] - per[1]
    assert inc1 > 0 and inc2 > 0
    assert inc2 < 2.0 * inc1, per          # linear growth per search would give 8x


# --------------------------------------------------------------------------- commit
def test_commit_matches_bruteforce_and_invariants():
    rng = np.random.default_rng(31)
    n = 300
    ty = (rng.random(n) < 0.2).astype(np.uint8)
    a = rng.integers(0, 4, size=n).astype(np.int32)
    ve = rng.integers(0, 3, size=n).astype(np.int32)
    vi = rng.integers(0, 3, size=n).astype(np.int32)
    off, src, elem = orc.search_list(a)
    # heavy collisions: targets drawn from 40 neurons, some -1
    tgt = rng.integers(0, 40, size=src.size)
    tgt[rng.random(src.size) < 0.1] = -1
    out = orc.commit(off, tgt, ty, a, ve, vi, 77, 3)
    acc = brute.commit_brute(off, tgt, ty, ve, vi, 77, 3)
    slots = np.nonzero(out["accepted"])[0]
    got = [(int(src[s]), int(elem[s])) for s in slots]
    assert got == acc
    assert np.array_equal(out["syn_src"], src[slots])
    assert np.array_equal(out["syn_tgt"], tgt[slots])
    assert np.array_equal(out["syn_type"], ty[src[slots]])
    assert out["n_formed"] == len(acc)
    # counts never negative; accepted <= vacant; accepted <= requests
    assert out["vac_exc"].min() >= 0 and out["vac_inh"].min() >= 0 and out["vac_axon"].min() >= 0
    for g in range(40):
        for t_ in (0, 1):
            req = int(((tgt == g) & (ty[src] == t_)).sum())
            vac = int((vi if t_ else ve)[g])
            took = vac - int((out["vac_inh"] if t_ else out["vac_exc"])[g])
            assert took == min(req, vac)
    # sorted by (src, elem)
    assert np.all(np.diff(out["syn_src"]) >= 0)
    assert np.array_equal(out["vac_axon"], a - np.bincount(out["syn_src"], minlength=n))


def test_commit_all_accepted_when_room():
    n = 50
    ty = np.zeros(n, np.uint8)
    a = np.ones(n, np.int32)
    off, src, elem = orc.search_list(a)
    tgt = (src + 1) % n
    out = orc.commit(off, tgt, ty, a, np.ones(n, np.int32), np.zeros(n, np.int32), 1, 0)
    assert out["n_formed"] == n
    assert np.all(out["vac_axon"] == 0) and np.all(out["vac_exc"] == 0)


def test_commit_acceptance_law():
    """10 requests on a neuron with 3 vacancies: each accepted w.p. 3/10."""
    from scipy import stats
    n = 11
    ty = np.zeros(n, np.uint8)
    a = np.ones(n, np.int32)
    a[0] = 0
    off, src, elem = orc.search_list(a)
    tgt = np.zeros(src.size, np.int64)
    ve = np.zeros(n, np.int32)
    ve[0] = 3
    wins = np.zeros(n, np.int64)
    steps = 4000
    for step in range(steps):
        out = orc.commit(off, tgt, ty, a, ve, np.zeros(n, np.int32), 5, step)
        assert out["n_formed"] == 3
        wins += np.bincount(out["syn_src"], minlength=n)
    p = stats.chisquare(wins[1:], np.full(10, steps * 0.3)).pvalue
    assert p > 1e-4, p


# --------------------------------------------------------------------------- attraction
def test_attraction_closed_form_two_neurons():
    pos = np.array([[100.0, 200.0, 300.0], [400.0, 250.0, 320.0]])
    t = orc.OracleTree(pos, np.zeros(3), 1000.0)
    t.update_counts(np.array([2, 3], np.int32), np.zeros(2, np.int32))
    ty = np.zeros(2, np.uint8)
    a = np.array([1, 0], np.int32)
    sigma = 350.0
    Z, L, dX, ds = t.attraction(ty, a, sigma, 0.3)
    d = pos[0] - pos[1]
    d2 = float(d @ d)
    assert Z[0] == pytest.approx(3.0 * math.exp(-d2 / sigma**2), rel=1e-15)
    assert L == pytest.approx(math.log(Z[0]), rel=1e-15)
    assert ds == pytest.approx(2 * d2 / sigma**3, rel=1e-13)
    assert np.allclose(dX[0], -2 * d / sigma**2, rtol=1e-13)
    assert np.allclose(dX[1], 2 * d / sigma**2, rtol=1e-13)


def test_attraction_theta0_direct_gradient():
    w = uniform_cube(200, 1000.0, seed=14)
    sigma = 400.0
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    Z, L, dX, ds = t.attraction(w.neuron_type, w.vac_axon, sigma, 0.0)
    # direct: Z_i = sum_{j != i} v_j^t exp(-|x_i - x_j|^2 / sigma^2) over type t = type_i
    X = w.pos
    D = X[:, None, :] - X[None, :, :]
    D2 = (D ** 2).sum(-1)
    V = np.where(w.neuron_type[:, None] == 1, w.vac_inh[None, :], w.vac_exc[None, :]).astype(float)
    np.fill_diagonal(V, 0.0)
    W = V * np.exp(-D2 / sigma**2)
    Zr = W.sum(1)
    src = w.vac_axon > 0
    assert np.allclose(Z[src], Zr[src], rtol=1e-12)
    Lr = np.log(Zr[src]).sum()
    assert L == pytest.approx(Lr, rel=1e-12)
    F = np.where(src[:, None], W / np.where(Zr > 0, Zr, 1)[:, None], 0.0)
    g_src = (F[:, :, None] * (-2 * D / sigma**2)).sum(1)
    g_tgt = (F[:, :, None] * (2 * D / sigma**2)).sum(0)
    assert np.allclose(dX, g_src + g_tgt, rtol=1e-9, atol=1e-12)
    dsr = (F * 2 * D2 / sigma**3).sum()
    assert ds == pytest.approx(dsr, rel=1e-10)


def test_attraction_finite_differences():
    w = uniform_cube(400, 1000.0, seed=15)
    sigma, theta = 350.0, 0.5
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    Z, L, dX, ds = t.attraction(w.neuron_type, w.vac_axon, sigma, theta)
    L0 = t.attraction_frozen(w.neuron_type, w.vac_axon, sigma, theta, w.pos)
    assert L0 == L
    h = 1e-3
    rng = np.random.default_rng(0)
    for _ in range(12):
        i, a = int(rng.integers(0, w.n)), int(rng.integers(0, 3))
        fd = t.frozen_derivative(w.neuron_type, w.vac_axon, sigma, theta, h, coord=(i, a))
        assert fd == pytest.approx(dX[i, a], rel=1e-6, abs=1e-12)
    fd = t.frozen_derivative(w.neuron_type, w.vac_axon, sigma, theta, h)
    assert fd == pytest.approx(ds, rel=1e-7)


# --------------------------------------------------------------------------- resume
def _run_updates(w, steps, state=None):
    a, e, i = (w.vac_axon.copy(), w.vac_exc.copy(), w.vac_inh.copy()) if state is None else state
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    syn = []
    for s in steps:
        t.update_counts(e, i)
        off, src, elem = orc.search_list(a)
        r = t.find_targets(w.neuron_type, w.sigma, w.theta, w.seed, s, src, elem)
        out = orc.commit(off, r["target"], w.neuron_type, a, e, i, w.seed, s)
        a, e, i = out["vac_axon"], out["vac_exc"], out["vac_inh"]
        syn.append((out["syn_src"], out["syn_tgt"], out["syn_type"]))
    return (a, e, i), syn


def test_checkpoint_resume_bitwise(tmp_path):
    w = uniform_cube(700, 1000.0, seed=19, a_hi=3, v_hi=2)
    full, syn_full = _run_updates(w, range(4))
    half, syn_a = _run_updates(w, range(2))
    np.savez(tmp_path / "ck.npz", a=half[0], e=half[1], i=half[2])
    ck = np.load(tmp_path / "ck.npz")
    rest, syn_b = _run_updates(w, range(2, 4), state=(ck["a"], ck["e"], ck["i"]))
    for x, y in zip(full, rest):
        assert np.array_equal(x, y)
    for x, y in zip(syn_full, syn_a + syn_b):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)
