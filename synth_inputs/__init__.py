"""Seeded synthetic inputs for the MSP connectivity update.

This module only draws random numbers: neuron positions, cell types and vacant
element counts in the shapes of the paper's workloads (synthetic networks that start
without connectivity, one to a few vacant elements per neuron; arXiv 2509.26193,
Sec. V-B), plus the host-side synaptic-element growth and deletion used between the
updates of the 100-update workload. It contains none of the octree, search or commit
arithmetic, and both the HIP library's tests and the oracle read inputs from here.

Every generator uses numpy.random.default_rng(seed) with a fixed draw order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    """One plain connectivity update: positions (um), types, vacant counts, parameters."""
    name: str
    pos: np.ndarray            # float64 [n, 3]
    box_min: np.ndarray        # float64 [3]
    box_edge: float
    neuron_type: np.ndarray    # uint8 [n], 0 = excitatory, 1 = inhibitory
    vac_axon: np.ndarray       # int32 [n]
    vac_exc: np.ndarray        # int32 [n], vacant excitatory dendritic elements
    vac_inh: np.ndarray        # int32 [n], vacant inhibitory dendritic elements
    sigma: float
    theta: float
    seed: int = 42
    step: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def searches(self) -> int:
        return int(np.maximum(self.vac_axon, 0).sum())


def _types(rng, n, frac_exc=0.8):
    """Exactly round(frac_exc * n) excitatory neurons, chosen by a permutation."""
    t = np.ones(n, dtype=np.uint8)
    t[rng.permutation(n)[: int(round(frac_exc * n))]] = 0
    return t


def _counts(rng, n, a_hi, v_hi):
    a = rng.integers(0, a_hi + 1, size=n, dtype=np.int64).astype(np.int32)
    e = rng.integers(0, v_hi + 1, size=n, dtype=np.int64).astype(np.int32)
    i = rng.integers(0, v_hi + 1, size=n, dtype=np.int64).astype(np.int32)
    return a, e, i


def bounding_cube(pos: np.ndarray):
    """Min corner and edge of the smallest axis-aligned cube holding every position."""
    mn = pos.min(axis=0)
    edge = float((pos.max(axis=0) - mn).max())
    if edge <= 0.0:
        edge = 1.0
    return mn.astype(np.float64), edge


def uniform_cube(n, edge, seed=42, a_hi=2, v_hi=3, sigma=750.0, theta=0.3, name=None):
    """n positions uniform in [0, edge)^3, 80/20 types, a ~ U{0..a_hi}, v ~ U{0..v_hi}."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, edge, size=(n, 3))
    t = _types(rng, n)
    a, e, i = _counts(rng, n, a_hi, v_hi)
    return Workload(name or f"uniform_{n}_{int(edge)}um", pos, np.zeros(3), float(edge), t, a, e,
                    i, float(sigma), float(theta), seed=seed)


def config_small(seed=42):
    """4096 neurons uniform in [0,1000)^3 um; sigma 750, theta 0.3."""
    return uniform_cube(4096, 1000.0, seed=seed, name="plain_4096_uniform_1000um")


def config_clusters(theta=0.3, seed=42, n_centres=64, per_centre=16384, std=150.0, edge=10000.0):
    """2^20 neurons in 64 isotropic Gaussian clusters (std 150 um), centres uniform in
    [0,10000)^3 um; cube = bounding cube of the sample; counts U{0..4}."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, edge, size=(n_centres, 3))
    n = n_centres * per_centre
    pos = np.repeat(centres, per_centre, axis=0) + rng.normal(0.0, std, size=(n, 3))
    t = _types(rng, n)
    a, e, i = _counts(rng, n, 4, 4)
    mn, L = bounding_cube(pos)
    return Workload(f"plain_{n}_clusters64_theta{theta}", pos, mn, L, t, a, e, i, 750.0,
                    float(theta), seed=seed)


def config_large(seed=42, n=1 << 23, edge=20000.0):
    """2^23 neurons uniform in [0,20000)^3 um, counts as the small case; theta 0.3."""
    return uniform_cube(n, edge, seed=seed, name=f"plain_{n}_uniform_{int(edge)}um")


def config_batched(seed=42, n_sims=64, log2_lo=12, log2_hi=18):
    """64 independent simulations, n_s log-uniform in [2^12, 2^18], cube edge scaled to
    the density of the 4096-neuron case, sigma_s ~ U[500, 1000] um, theta 0.3."""
    rng = np.random.default_rng(seed)
    u = rng.random(n_sims)
    ns = np.clip(np.round(2.0 ** (log2_lo + (log2_hi - log2_lo) * u)), 2 ** log2_lo,
                 2 ** log2_hi).astype(np.int64)
    sims = []
    for s in range(n_sims):
        n = int(ns[s])
        edge = 1000.0 * (n / 4096.0) ** (1.0 / 3.0)
        pos = rng.uniform(0.0, edge, size=(n, 3))
        sigma = float(rng.uniform(500.0, 1000.0))
        t = _types(rng, n)
        a, e, i = _counts(rng, n, 2, 3)
        sims.append(Workload(f"sim{s}_{n}", pos, np.zeros(3), edge, t, a, e, i, sigma, 0.3,
                             seed=seed))
    return sims


def config_attraction(seed=42):
    """262144 neurons uniform in [0,5000)^3 um, sigma 750, theta 0.3."""
    return uniform_cube(262144, 5000.0, seed=seed, name="attraction_262144_uniform_5000um")


# ---------------------------------------------------------------------------
# Host-side plasticity between updates of the 100-update workload (input generation
# for the next update; not part of the connectivity update itself).
# Synaptic-element growth: dz = nu * (2 exp(-((Ca - xi)/zeta)^2) - 1) per step, with
# target eps = 0.7 and growth rate nu = 0.001 (Sec. V-D), growth onset eta = 0.4;
# xi = (eta + eps) / 2, zeta = (eps - eta) / (2 sqrt(ln 2)); applied for the 100 steps
# between two connectivity updates.
# ---------------------------------------------------------------------------
def growth_delta(ca, nu=0.001, eps=0.7, eta=0.4, steps=100):
    xi = 0.5 * (eta + eps)
    zeta = (eps - eta) / (2.0 * np.sqrt(np.log(2.0)))
    return steps * nu * (2.0 * np.exp(-((ca - xi) / zeta) ** 2) - 1.0)


@dataclass
class PlasticityState:
    """Continuous element counts z (axon, exc dendrite, inh dendrite) and bound synapses."""
    z: np.ndarray              # float64 [3, n]
    bound: np.ndarray          # int64 [3, n] elements bound in synapses
    syn_src: np.ndarray        # int64 [m]
    syn_tgt: np.ndarray        # int64 [m]
    syn_type: np.ndarray       # uint8 [m]

    def copy(self) -> "PlasticityState":
        return PlasticityState(self.z.copy(), self.bound.copy(), self.syn_src.copy(),
                               self.syn_tgt.copy(), self.syn_type.copy())

    def save(self, path) -> None:
        np.savez(path, z=self.z, bound=self.bound, syn_src=self.syn_src, syn_tgt=self.syn_tgt,
                 syn_type=self.syn_type)

    @staticmethod
    def load(path) -> "PlasticityState":
        with np.load(path) as f:
            return PlasticityState(f["z"], f["bound"], f["syn_src"], f["syn_tgt"], f["syn_type"])


def plasticity_init(w: Workload) -> PlasticityState:
    z = np.stack([w.vac_axon, w.vac_exc, w.vac_inh]).astype(np.float64)
    return PlasticityState(z, np.zeros((3, w.n), np.int64), np.zeros(0, np.int64),
                           np.zeros(0, np.int64), np.zeros(0, np.uint8))


def _unbind(state: PlasticityState, gone: np.ndarray) -> None:
    """Remove the synapses flagged in `gone`: each frees one axonal element of its
    source and one dendritic element (of the synapse's type) of its target."""
    if not gone.any():
        return
    n = state.z.shape[1]
    state.bound[0] -= np.bincount(state.syn_src[gone], minlength=n)
    ty = state.syn_type[gone]
    tg = state.syn_tgt[gone]
    state.bound[1] -= np.bincount(tg[ty == 0], minlength=n)
    state.bound[2] -= np.bincount(tg[ty == 1], minlength=n)
    keep = ~gone
    state.syn_src, state.syn_tgt, state.syn_type = (state.syn_src[keep], state.syn_tgt[keep],
                                                    state.syn_type[keep])


def plasticity_step(state: PlasticityState, neuron_type, seed: int, step: int, delete_frac=0.1):
    """Host-side change of the network between update `step` and the next: Ca ~
    N(0.7, 0.1) per neuron and element kind, growth/retraction of the continuous element
    counts, deletion of 10 % of the synapses at random, then retraction of bound
    elements where a count fell below the bound ones (random synapses of that neuron
    break). Returns the vacant counts (axon, exc, inh) as int32 for the next update.

    The random numbers come from a generator seeded by (seed, step) alone, so a run
    resumed from a saved state continues exactly as an uninterrupted one."""
    rng = np.random.default_rng([int(seed), 0x5EED, int(step)])
    n = state.z.shape[1]
    ca = rng.normal(0.7, 0.1, size=(3, n))
    state.z = np.maximum(state.z + growth_delta(ca), 0.0)
    m = state.syn_src.size
    gone = np.zeros(m, dtype=bool)
    n_del = int(round(delete_frac * m))
    if n_del > 0:
        gone[rng.choice(m, size=n_del, replace=False)] = True
    _unbind(state, gone)
    cap = np.floor(state.z).astype(np.int64)
    for kind in range(3):
        excess = state.bound[kind] - cap[kind]
        if not (excess > 0).any():
            continue
        owner = state.syn_src if kind == 0 else state.syn_tgt
        sel = excess[owner] > 0
        if kind > 0:
            sel &= state.syn_type == kind - 1
        idx = np.nonzero(sel)[0]
        pri = rng.random(idx.size)
        o = np.lexsort((pri, owner[idx]))          # by owner, then random priority
        idx = idx[o]
        own = owner[idx]
        start = np.r_[0, np.nonzero(own[1:] != own[:-1])[0] + 1]
        rank = np.arange(own.size) - np.repeat(start, np.diff(np.r_[start, own.size]))
        gone = np.zeros(state.syn_src.size, dtype=bool)
        gone[idx[rank < excess[own]]] = True
        _unbind(state, gone)
    vac = np.maximum(np.floor(state.z).astype(np.int64) - state.bound, 0).astype(np.int32)
    return vac[0].copy(), vac[1].copy(), vac[2].copy()


def plasticity_record(state: PlasticityState, syn_src, syn_tgt, syn_type):
    """Add newly formed synapses to the host state."""
    n = state.z.shape[1]
    syn_src = np.asarray(syn_src, np.int64)
    syn_tgt = np.asarray(syn_tgt, np.int64)
    syn_type = np.asarray(syn_type, np.uint8)
    state.bound[0] += np.bincount(syn_src, minlength=n)
    state.bound[1] += np.bincount(syn_tgt[syn_type == 0], minlength=n)
    state.bound[2] += np.bincount(syn_tgt[syn_type == 1], minlength=n)
    state.syn_src = np.concatenate([state.syn_src, syn_src])
    state.syn_tgt = np.concatenate([state.syn_tgt, syn_tgt])
    state.syn_type = np.concatenate([state.syn_type, syn_type])
