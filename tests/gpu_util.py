"""Helpers shared by the GPU parity tests: run the HIP path and compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

import paper_2509_26193_amd as msp
from oracle import oracle as orc

DEV = torch.device("cuda:0")
Z_REL_TOL = 1e-5          # float32 kernel sums vs the float64 oracle
WINDOW = 1e-6             # a differing choice must lie within this CDF distance
MAX_DIFF_SHARE = 1e-4     # share of searches whose choice differs


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def T(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


def gpu_search(w, theta=None, sigma=None, step=None, seed=None):
    """Build + refresh + search on the GPU. Returns a dict of host arrays and the tree."""
    theta = w.theta if theta is None else theta
    sigma = w.sigma if sigma is None else sigma
    step = w.step if step is None else step
    seed = w.seed if seed is None else seed
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    ve, vi = T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32)
    msp.update_vacant_counts(tree, ve, vi)
    ty, va = T(w.neuron_type, torch.uint8), T(w.vac_axon, torch.int32)
    tgt, off, z0, lv, cnt = msp.find_targets(tree, ty, va, sigma, theta, seed, step, diag=True,
                                             counters=True)
    torch.cuda.synchronize()
    return dict(tree=tree, target=tgt.cpu().numpy().astype(np.int64), off=off.cpu().numpy(),
                z0=z0.cpu().numpy(), levels=lv.cpu().numpy(), ty=ty, va=va, ve=ve, vi=vi,
                visits=cnt["visits"].cpu().numpy(), opens=cnt["opens"].cpu().numpy(),
                visits0=cnt["visits0"].cpu().numpy(), opens0=cnt["opens0"].cpu().numpy(),
                entries0=cnt["entries0"].cpu().numpy())


def oracle_tree(w):
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    return t


def compare_search(g_target, g_z0, o, label=""):
    """Targets identical except inside boundary windows; z0 within the tolerance."""
    diff = g_target != o["target"]
    nd = int(diff.sum())
    outside = diff & ~(o["window"] < WINDOW)
    share = nd / max(1, diff.size)
    pos = o["z0"] > 0
    rel = np.abs(g_z0[pos] - o["z0"][pos]) / o["z0"][pos]
    zero_mismatch = int(((g_z0 > 0) != pos).sum())
    say(f"[{label}] searches={diff.size} differing={nd} (share {share:.2e}) "
        f"outside-window={int(outside.sum())} max-rel-z0={rel.max() if rel.size else 0:.2e} "
        f"z0-zero-mismatch={zero_mismatch}")
    assert int(outside.sum()) == 0, np.nonzero(outside)[0][:10]
    assert share < MAX_DIFF_SHARE or nd <= 1
    assert zero_mismatch == 0
    if rel.size:
        assert rel.max() < Z_REL_TOL
    return nd


def compare_targets(g_target, o, label=""):
    """Targets identical except inside boundary windows (no normaliser to compare)."""
    diff = g_target != o["target"]
    nd = int(diff.sum())
    outside = diff & ~(o["window"] < WINDOW)
    say(f"[{label}] searches={diff.size} differing={nd} outside-window={int(outside.sum())}")
    assert int(outside.sum()) == 0, np.nonzero(outside)[0][:10]
    assert nd / max(1, diff.size) < MAX_DIFF_SHARE or nd <= 1
    return nd
