"""Seeded synthetic inputs for the MSP connectivity update.

This module only draws random numbers: neuron positions, cell types and vacant
element counts in the shapes of the paper's workloads (synthetic networks that start
without connectivity, one to a few vacant elements per neuron; arXiv 2509.26193,
Sec. V-B). It contains none of the octree, search, commit or plasticity arithmetic,
and both the HIP library's tests and the oracle read inputs from here.

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
