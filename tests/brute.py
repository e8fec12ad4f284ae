"""Independent pure-Python references used to pin the oracle on tiny inputs.

Nothing here imports the oracle or the HIP library. The octree is built by inserting
points one at a time (cell splitting), which is a different construction from the
oracle's recursive split of a sorted range; the search list, the theta = 0 brute force
and the exact implied target distribution are written from the paper's description
(arXiv 2509.26193, Sec. II and Sec. III-B, "Division of work").
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def fma(a: float, b: float, c: float) -> float:
    """a * b + c rounded once (exact rational arithmetic, then one rounding)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def sqdist(dx: float, dy: float, dz: float) -> float:
    """dx^2 + dy^2 + dz^2 with the last two terms fused, as the method's reading fixes."""
    return fma(dz, dz, fma(dy, dy, dx * dx))

DEPTH = 21
CELLS = 2097152.0  # 2^21


def philox_u(seed, stream, ctr):
    """u = top 24 bits of Philox4x64-10 word 0 for counter ctr (numpy's generator).

    numpy's Philox advances the counter before producing a block, so the block for
    counter c is produced by a generator started at c - 1 (256-bit little endian)."""
    c = ctr[0] | (ctr[1] << 64) | (ctr[2] << 128) | (ctr[3] << 192)
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * k)) & ((1 << 64) - 1) for k in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([seed, stream], dtype=np.uint64), counter=words)
    r = int(bg.random_raw(1)[0])
    return (r >> 40) * 2.0 ** -24, r


def quantise(x, x0, L):
    f = math.floor(((x - x0) / L) * CELLS)
    return int(min(max(f, 0.0), CELLS - 1.0))


def digits(q):
    """Octant digits at depths 1..21: 4*x_bit + 2*y_bit + z_bit, most significant first."""
    qx, qy, qz = q
    return [(((qx >> (DEPTH - k)) & 1) << 2) | (((qy >> (DEPTH - k)) & 1) << 1)
            | ((qz >> (DEPTH - k)) & 1) for k in range(1, DEPTH + 1)]


class Cell:
    __slots__ = ("depth", "path", "kids", "members")

    def __init__(self, depth, path):
        self.depth = depth
        self.path = path          # digits from the root
        self.kids = {}            # digit -> Cell (inner)
        self.members = []         # neuron ids (leaf)

    @property
    def leaf(self):
        return not self.kids


class InsertTree:
    """Octree by insertion: a leaf that receives a second neuron splits into octants,
    until depth 21, where coincident quantised neurons share a bucket leaf."""

    def __init__(self, pos, x0, L):
        self.pos = [tuple(float(c) for c in p) for p in pos]
        self.L = float(L)
        self.dig = [digits(tuple(quantise(p[a], x0[a], L) for a in range(3))) for p in self.pos]
        self.root = Cell(0, ())
        for i in range(len(self.pos)):
            self._insert(i)

    def _insert(self, i):
        c = self.root
        while True:
            if c.leaf:
                if not c.members or c.depth == DEPTH:
                    c.members.append(i)
                    return
                # split: push the resident neuron(s) one level down
                old = c.members
                c.members = []
                for j in old:
                    d = self.dig[j][c.depth]
                    child = c.kids.setdefault(d, Cell(c.depth + 1, c.path + (d,)))
                    child.members.append(j)
                # continue inserting i below (may split again)
            d = self.dig[i][c.depth]
            if d not in c.kids:
                c.kids[d] = Cell(c.depth + 1, c.path + (d,))
                c.kids[d].members.append(i)
                return
            c = c.kids[d]

    def preorder(self):
        out = []

        def rec(c):
            out.append(c)
            for d in sorted(c.kids):
                rec(c.kids[d])
        rec(self.root)
        return out

    def leaves_in_order(self, c):
        """Neuron ids below c in digit order, bucket members in id order."""
        if c.leaf:
            return sorted(c.members)
        out = []
        for d in sorted(c.kids):
            out.extend(self.leaves_in_order(c.kids[d]))
        return out

    def aggregate(self, vac):
        """vac: list of per-neuron counts of one type. Returns {id(cell): (v, (x, y, z))}."""
        agg = {}

        def rec(c):
            if c.leaf:
                if len(c.members) == 1:
                    j = c.members[0]
                    agg[id(c)] = (vac[j], self.pos[j])
                    return agg[id(c)]
                v = 0
                s = [0.0, 0.0, 0.0]
                for j in sorted(c.members):
                    v += vac[j]
                    if vac[j] > 0:
                        for a in range(3):
                            s[a] = s[a] + float(vac[j]) * self.pos[j][a]
                cen = tuple(s[a] / float(v) for a in range(3)) if v > 0 else (0.0, 0.0, 0.0)
                agg[id(c)] = (v, cen)
                return agg[id(c)]
            v = 0
            s = [0.0, 0.0, 0.0]
            for d in sorted(c.kids):
                vk, ck = rec(c.kids[d])
                v += vk
                if vk > 0:
                    for a in range(3):
                        s[a] = s[a] + float(vk) * ck[a]
            cen = tuple(s[a] / float(v) for a in range(3)) if v > 0 else (0.0, 0.0, 0.0)
            agg[id(c)] = (v, cen)
            return agg[id(c)]
        rec(self.root)
        return agg

    def contains(self, c, i):
        return tuple(self.dig[i][: c.depth]) == c.path

    def bh_list(self, agg, vac, i, start, sigma, theta):
        """Accepted list of the expansion of `start` for source i: [(kind, obj, w)],
        kind 'n' = neuron id, 'c' = cell. The start cell is always opened; leaves are
        always accepted; own cell opened; otherwise accept iff l^2 < theta^2 d^2."""
        xi = self.pos[i]
        out = []

        def weight(v, c):
            dx = xi[0] - c[0]
            dy = xi[1] - c[1]
            dz = xi[2] - c[2]
            d2 = sqdist(dx, dy, dz)
            return float(v) * math.exp(-(d2 / (sigma * sigma))), d2

        def leaf_members(c):
            for j in sorted(c.members):
                if j != i and vac[j] > 0:
                    out.append(("n", j, weight(vac[j], self.pos[j])[0]))

        def visit(c):
            v, cen = agg[id(c)]
            if v == 0:
                return
            if c.leaf:
                leaf_members(c)
                return
            if self.contains(c, i):
                op = True
            else:
                _, d2 = weight(v, cen)
                l = math.ldexp(self.L, -c.depth)
                op = not (l * l < (theta * theta) * d2)
            if not op:
                out.append(("c", c, weight(v, cen)[0]))
                return
            for d in sorted(c.kids):
                visit(c.kids[d])

        if start.leaf:
            if agg[id(start)][0] > 0:
                leaf_members(start)
        else:
            for d in sorted(start.kids):
                visit(start.kids[d])
        return out

    def search(self, agg, vac, i, j, sigma, theta, seed, step):
        """One search with the inverse-CDF draw and restarts. Returns (target, Z0)."""
        S = self.root
        z0 = None
        for level in range(64):
            lst = self.bh_list(agg, vac, i, S, sigma, theta)
            Z = 0.0
            for e in lst:
                Z = Z + e[2]
            if z0 is None:
                z0 = Z
            if not lst or Z == 0.0:
                return -1, z0
            u, _ = philox_u(seed, 0, (i, j, step, level))
            T = u * Z
            P = 0.0
            ch = None
            for e in lst:
                P = P + e[2]
                if P > T:
                    ch = e
                    break
            if ch is None:
                ch = [e for e in lst if e[2] > 0.0][-1]
            if ch[0] == "n":
                return ch[1], z0
            S = ch[1]
        raise RuntimeError("restart chain longer than the tree depth")

    def bh_list_counted(self, agg, vac, i, start, sigma, theta):
        """bh_list with the work of the expansion counted, written out separately:
        node records examined (the start node once, every node reached below it,
        skipped ones included, a bucket leaf once) and nodes replaced by their
        children (the start node included when it is inner)."""
        xi = self.pos[i]
        out = []
        cnt = [0, 0]                      # visits, opens

        def w_of(v, c):
            d2 = sqdist(xi[0] - c[0], xi[1] - c[1], xi[2] - c[2])
            return float(v) * math.exp(-(d2 / (sigma * sigma))), d2

        def members(c):
            for j in sorted(c.members):
                if j != i and vac[j] > 0:
                    out.append(("n", j, w_of(vac[j], self.pos[j])[0]))

        def visit(c):
            cnt[0] += 1
            v, cen = agg[id(c)]
            if v == 0:
                return
            if c.leaf:
                members(c)
                return
            if self.contains(c, i):
                op = True
            else:
                l = math.ldexp(self.L, -c.depth)
                op = not (l * l < (theta * theta) * w_of(v, cen)[1])
            if not op:
                out.append(("c", c, w_of(v, cen)[0]))
                return
            cnt[1] += 1
            for d in sorted(c.kids):
                visit(c.kids[d])

        cnt[0] += 1
        if start.leaf:
            if agg[id(start)][0] > 0:
                members(start)
        else:
            cnt[1] += 1
            for d in sorted(start.kids):
                visit(start.kids[d])
        return out, cnt[0], cnt[1]

    def search_full(self, agg, vac, i, j, sigma, theta, seed, step):
        """One search with every per-search output of the method's checker: target,
        level-0 normaliser and the length of the level-0 list, the levels drawn, the node
        records examined and the nodes opened over all levels, and the boundary
        distance of the draw: at each level
        the chosen entry covers [P_prev / Z, P / Z) of the cumulative distribution
        (running sums in list order), its distance is min(u - P_prev / Z, P / Z - u),
        and the search's is the smallest over its levels (1 if it never draws).
        Returns a dict, and for each level the exact rational bounds of the chosen
        entry (Fractions of the same float weights) so that callers can check the
        float distance against exact arithmetic."""
        S = self.root
        res = dict(target=-1, z0=None, window=1.0, levels=0, visits=0, opens=0, entries0=0)
        exact = []
        for level in range(64):
            lst, nv, no = self.bh_list_counted(agg, vac, i, S, sigma, theta)
            res["visits"] += nv
            res["opens"] += no
            res["levels"] += 1
            Z = 0.0
            for e in lst:
                Z = Z + e[2]
            if res["z0"] is None:
                res["z0"] = Z
                res["entries0"] = len(lst)
            if not lst or Z == 0.0:
                res["target"] = -1
                return res, exact
            u, _ = philox_u(seed, 0, (i, j, step, level))
            T = u * Z
            P = 0.0
            k = None
            prefix = []
            for n_, e in enumerate(lst):
                prev = P
                P = P + e[2]
                prefix.append((prev, P))
                if P > T:
                    k = n_
                    break
            if k is None:                     # rounding: the last entry with weight
                k = max(n_ for n_, e in enumerate(lst) if e[2] > 0.0)
                lo = hi = Z
            else:
                lo, hi = prefix[k]
            res["window"] = min(res["window"], min(abs(u - lo / Z), abs(hi / Z - u)))
            ws = [Fraction(e[2]) for e in lst]
            Ze = sum(ws, Fraction(0))
            exact.append((Fraction(u), sum(ws[:k], Fraction(0)) / Ze,
                          sum(ws[:k + 1], Fraction(0)) / Ze))
            ch = lst[k]
            if ch[0] == "n":
                res["target"] = ch[1]
                return res, exact
            S = ch[1]
        raise RuntimeError("restart chain longer than the tree depth")

    def implied_distribution(self, agg, vac, i, sigma, theta):
        """Exact P(target = g | source i) of the restart process, as a dict; the mass
        of 'no target' is under key -1."""
        dist = {}

        def rec(S, mass):
            lst = self.bh_list(agg, vac, i, S, sigma, theta)
            Z = math.fsum(e[2] for e in lst)
            if not lst or Z == 0.0:
                dist[-1] = dist.get(-1, 0.0) + mass
                return
            for kind, obj, w in lst:
                p = mass * w / Z
                if p == 0.0:
                    continue
                if kind == "n":
                    dist[obj] = dist.get(obj, 0.0) + p
                else:
                    rec(obj, p)
        rec(self.root, 1.0)
        return dist


def brute_theta0(pos, order, vac, i, j, sigma, seed, step):
    """Direct O(n) search for one element at theta = 0: every other neuron with a
    vacancy, in (key, id) order, weight v * exp(-d^2 / sigma^2); one draw."""
    xi = pos[i]
    ws = []
    ids = []
    for g in order:
        g = int(g)
        if g == i or vac[g] <= 0:
            continue
        dx = float(xi[0]) - float(pos[g][0])
        dy = float(xi[1]) - float(pos[g][1])
        dz = float(xi[2]) - float(pos[g][2])
        d2 = sqdist(dx, dy, dz)
        ws.append(float(vac[g]) * math.exp(-(d2 / (sigma * sigma))))
        ids.append(g)
    Z = 0.0
    for w in ws:
        Z = Z + w
    if not ws or Z == 0.0:
        return -1, Z
    u, _ = philox_u(seed, 0, (i, j, step, 0))
    T = u * Z
    P = 0.0
    for g, w in zip(ids, ws):
        P = P + w
        if P > T:
            return g, Z
    return [g for g, w in zip(ids, ws) if w > 0][-1], Z


def commit_brute(elem_offset, target, neuron_type, vac_exc, vac_inh, seed, step):
    """Random acceptance by sorting each (target, type) group on the Philox stream-1
    priority with ties broken by (i, j). Returns the sorted (i, j) pairs accepted."""
    groups = {}
    n = len(elem_offset) - 1
    for i in range(n):
        for s in range(int(elem_offset[i]), int(elem_offset[i + 1])):
            g = int(target[s])
            if g < 0:
                continue
            j = s - int(elem_offset[i])
            _, prio = philox_u(seed, 1, (i, j, step, 0))
            groups.setdefault((g, int(neuron_type[i])), []).append((prio, i, j))
    acc = []
    for (g, ty), reqs in groups.items():
        vac = int(vac_inh[g] if ty else vac_exc[g])
        reqs.sort()
        acc.extend((i, j) for _, i, j in reqs[:vac])
    return sorted(acc)
