"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the fp64 CPU oracle (msp_oracle.cpp).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
module. It shares no code with the HIP library and never imports it.

The oracle follows the MSP connectivity update of arXiv 2509.26193: the octree and
its vacancy aggregates (Sec. III-B, "Spatial octree" and "Division of work"), the
Barnes-Hut target search with restarts (Sec. III-B, "Division of work"; Sec. II for
theta = 0), the random acceptance of requests (Sec. III-A, "Update of synapses"), the
expected-attraction adjoint used by the differentiated form, and the growth and
deletion of synaptic elements between updates (Sec. III-A).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msp_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "libmsp_oracle.so")

_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_dbl = ctypes.c_double
_ptr = ctypes.c_void_p


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with g++ (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", _SRC, "-o", _LIB_PATH + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    """The oracle library: built here on first use, or, when MSP_ORACLE_LIB names a
    prebuilt one (the sanitizer test's instrumented build of the same source), that."""
    global _lib
    if _lib is None:
        path = os.environ.get("MSP_ORACLE_LIB") or build_oracle()
        L = ctypes.CDLL(path)
        L.oracle_build.restype = _ptr
        L.oracle_build.argtypes = [_ptr, _i64, _ptr, _dbl]
        L.oracle_free.argtypes = [_ptr]
        L.oracle_num_nodes.restype = _i64
        L.oracle_num_nodes.argtypes = [_ptr]
        L.oracle_get_order.argtypes = [_ptr, _ptr, _ptr]
        L.oracle_get_nodes.argtypes = [_ptr, _ptr, _ptr, _ptr, _ptr, _ptr]
        L.oracle_update_counts.restype = ctypes.c_int
        L.oracle_update_counts.argtypes = [_ptr, _ptr, _ptr]
        L.oracle_get_aggregates.argtypes = [_ptr, ctypes.c_int, _ptr, _ptr]
        L.oracle_find_targets.restype = ctypes.c_int
        L.oracle_find_targets.argtypes = [_ptr, _ptr, _dbl, _dbl, _u64, _u64, _ptr, _ptr, _i64,
                                          _ptr, _ptr, _ptr, _ptr, _ptr, _ptr, _ptr, ctypes.c_int]
        L.oracle_commit.restype = _i64
        L.oracle_commit.argtypes = [_i64, _ptr, _ptr, _ptr, _ptr, _ptr, _ptr, _u64, _u64,
                                    _ptr, _ptr, _ptr, _ptr]
        L.oracle_philox4x64_10.argtypes = [_ptr, _ptr, _ptr]
        L.oracle_attraction.restype = ctypes.c_int
        L.oracle_attraction.argtypes = [_ptr, _ptr, _ptr, _dbl, _dbl, _ptr, _ptr, _ptr, _ptr,
                                        ctypes.c_int]
        L.oracle_attraction_frozen.restype = _dbl
        L.oracle_attraction_frozen.argtypes = [_ptr, _ptr, _ptr, _dbl, _dbl, _ptr, _ptr,
                                               ctypes.c_int]
        L.oracle_growth_delta.restype = _dbl
        L.oracle_growth_delta.argtypes = [_dbl, _dbl, _dbl, _dbl, ctypes.c_int32]
        L.oracle_calcium.restype = _dbl
        L.oracle_calcium.argtypes = [_u64, _u64, _u64, _u64, _dbl, _dbl]
        L.oracle_plasticity_record.argtypes = [_i64, _i64, _i64, _ptr, _ptr, _ptr, _ptr, _ptr,
                                               _ptr, _ptr]
        L.oracle_plasticity_step.restype = _i64
        L.oracle_plasticity_step.argtypes = [_i64, _i64, _dbl, _dbl, _dbl, ctypes.c_int32, _dbl,
                                             _dbl, _dbl, _u64, _u64, _ptr, _ptr, _ptr, _ptr,
                                             _ptr, _ptr]
        L.oracle_activity_run.restype = _i64
        L.oracle_activity_run.argtypes = [_i64, _ptr, _ptr, _i64, _ptr, _ptr, _ptr,
                                          ctypes.c_int32, _ptr, _dbl, _dbl, ctypes.c_int32,
                                          _u64, _u64, ctypes.c_int32, _ptr, _ptr, _ptr, _ptr,
                                          _ptr, _ptr, _ptr]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_ptr) if a is not None else None


def philox4x64_10(ctr, key) -> np.ndarray:
    """One Philox4x64-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().oracle_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def search_list(vac_axon: np.ndarray):
    """CSR of searches: elem_offset[n+1], and the (source, element) of every search."""
    a = np.asarray(vac_axon, dtype=np.int64)
    off = np.zeros(a.size + 1, dtype=np.int64)
    np.cumsum(np.maximum(a, 0), out=off[1:])
    src = np.repeat(np.arange(a.size, dtype=np.int64), np.maximum(a, 0))
    elem = np.arange(off[-1], dtype=np.int64) - off[src]
    return off, src, elem


class OracleTree:
    """Octree over fixed neuron positions, with per-type vacancy aggregates."""

    def __init__(self, pos: np.ndarray, box_min, box_edge: float):
        self.pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        self.n = self.pos.shape[0]
        bm = np.ascontiguousarray(box_min, dtype=np.float64)
        h = lib().oracle_build(_p(self.pos), self.n, _p(bm), float(box_edge))
        if not h:
            raise ValueError("oracle_build rejected the input")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_free(h)
            self._h = None

    @property
    def num_nodes(self) -> int:
        return int(lib().oracle_num_nodes(self._h))

    def order(self):
        order = np.zeros(self.n, dtype=np.int64)
        keys = np.zeros(self.n, dtype=np.uint64)
        lib().oracle_get_order(self._h, _p(order), _p(keys))
        return order, keys

    def nodes(self) -> dict:
        N = self.num_nodes
        d = dict(depth=np.zeros(N, np.int32), begin=np.zeros(N, np.int64),
                 end=np.zeros(N, np.int64), subtree_end=np.zeros(N, np.int64),
                 is_leaf=np.zeros(N, np.uint8))
        lib().oracle_get_nodes(self._h, _p(d["depth"]), _p(d["begin"]), _p(d["end"]),
                               _p(d["subtree_end"]), _p(d["is_leaf"]))
        return d

    def update_counts(self, vac_exc, vac_inh) -> None:
        e = np.ascontiguousarray(vac_exc, dtype=np.int32)
        i = np.ascontiguousarray(vac_inh, dtype=np.int32)
        if lib().oracle_update_counts(self._h, _p(e), _p(i)) != 0:
            raise ValueError("negative vacancy count")

    def aggregates(self, type_: int):
        N = self.num_nodes
        v = np.zeros(N, np.int64)
        c = np.zeros((N, 3), np.float64)
        lib().oracle_get_aggregates(self._h, int(type_), _p(v), _p(c))
        return v, c

    def find_targets(self, neuron_type, sigma, theta, seed, step, src, elem, nthreads=0) -> dict:
        t = np.ascontiguousarray(neuron_type, dtype=np.uint8)
        src = np.ascontiguousarray(src, dtype=np.int64)
        elem = np.ascontiguousarray(elem, dtype=np.int64)
        m = src.size
        out = dict(target=np.zeros(m, np.int64), z0=np.zeros(m, np.float64),
                   window=np.zeros(m, np.float64), levels=np.zeros(m, np.int32),
                   visits=np.zeros(m, np.int64), opens=np.zeros(m, np.int64),
                   entries0=np.zeros(m, np.int64))
        rc = lib().oracle_find_targets(self._h, _p(t), float(sigma), float(theta), int(seed),
                                       int(step), _p(src), _p(elem), m, _p(out["target"]),
                                       _p(out["z0"]), _p(out["window"]), _p(out["levels"]),
                                       _p(out["visits"]), _p(out["opens"]),
                                       _p(out["entries0"]), int(nthreads))
        if rc != 0:
            raise ValueError("oracle_find_targets rejected the input")
        return out

    def attraction(self, neuron_type, vac_axon, sigma, theta, nthreads=0):
        t = np.ascontiguousarray(neuron_type, dtype=np.uint8)
        a = np.ascontiguousarray(vac_axon, dtype=np.int32)
        Z = np.zeros(self.n, np.float64)
        dX = np.zeros((self.n, 3), np.float64)
        L = np.zeros(1, np.float64)
        ds = np.zeros(1, np.float64)
        rc = lib().oracle_attraction(self._h, _p(t), _p(a), float(sigma), float(theta), _p(Z),
                                     _p(L), _p(dX), _p(ds), int(nthreads))
        if rc != 0:
            raise ValueError("oracle_attraction rejected the input")
        return Z, float(L[0]), dX, float(ds[0])

    def attraction_frozen(self, neuron_type, vac_axon, sigma, theta, pos_new, nthreads=0,
                          return_z=False):
        """L (and, with return_z, every Z_i) at positions pos_new / width sigma with the
        accepted sets of the tree's own geometry."""
        t = np.ascontiguousarray(neuron_type, dtype=np.uint8)
        a = np.ascontiguousarray(vac_axon, dtype=np.int32)
        p = np.ascontiguousarray(pos_new, dtype=np.float64)
        Z = np.zeros(self.n, np.float64) if return_z else None
        L = float(lib().oracle_attraction_frozen(self._h, _p(t), _p(a), float(sigma),
                                                 float(theta), _p(p), _p(Z), int(nthreads)))
        return (L, Z) if return_z else L

    def frozen_derivative(self, neuron_type, vac_axon, sigma, theta, h, coord=None,
                          nthreads=0):
        """Central difference of L = sum_i log Z_i in one position coordinate
        coord = (i, axis), or in sigma if coord is None, with frozen sets. The
        difference is summed per source as log1p((Z+ - Z-) / Z-), which keeps its
        precision where L itself is large."""
        if coord is None:
            _, zp = self.attraction_frozen(neuron_type, vac_axon, sigma + h, theta, self.pos,
                                           nthreads, True)
            _, zm = self.attraction_frozen(neuron_type, vac_axon, sigma - h, theta, self.pos,
                                           nthreads, True)
        else:
            i, ax = coord
            p = self.pos.copy()
            p[i, ax] += h
            _, zp = self.attraction_frozen(neuron_type, vac_axon, sigma, theta, p, nthreads, True)
            p[i, ax] -= 2 * h
            _, zm = self.attraction_frozen(neuron_type, vac_axon, sigma, theta, p, nthreads, True)
        ok = (zp > 0) & (zm > 0)
        return float(np.sum(np.log1p((zp[ok] - zm[ok]) / zm[ok]))) / (2 * h)


def commit(elem_offset, target, neuron_type, vac_axon, vac_exc, vac_inh, seed, step):
    """Random acceptance of all requests. Returns synapses and the updated counts."""
    off = np.ascontiguousarray(elem_offset, dtype=np.int64)
    tg = np.ascontiguousarray(target, dtype=np.int64)
    ty = np.ascontiguousarray(neuron_type, dtype=np.uint8)
    a = np.array(vac_axon, dtype=np.int32, copy=True)
    e = np.array(vac_exc, dtype=np.int32, copy=True)
    i = np.array(vac_inh, dtype=np.int32, copy=True)
    S = int(off[-1])
    ss = np.zeros(max(S, 1), np.int64)
    st = np.zeros(max(S, 1), np.int64)
    sy = np.zeros(max(S, 1), np.uint8)
    acc = np.zeros(max(S, 1), np.uint8)
    m = int(lib().oracle_commit(a.size, _p(off), _p(tg), _p(ty), _p(a), _p(e), _p(i), int(seed),
                                int(step), _p(ss), _p(st), _p(sy), _p(acc)))
    return dict(syn_src=ss[:m].copy(), syn_tgt=st[:m].copy(), syn_type=sy[:m].copy(),
                vac_axon=a, vac_exc=e, vac_inh=i, n_formed=m, accepted=acc[:S].copy())


# --------------------------------------------------------------------------- plasticity
PLASTICITY = dict(nu=0.001, eps=0.7, eta=0.4, steps=100, ca_mean=0.7, ca_sd=0.1,
                  delete_frac=0.1)


def growth_delta(ca: float, nu=0.001, eps=0.7, eta=0.4, steps=100) -> float:
    return float(lib().oracle_growth_delta(float(ca), nu, eps, eta, int(steps)))


def calcium(seed: int, j: int, k: int, step: int, mean=0.7, sd=0.1) -> float:
    return float(lib().oracle_calcium(int(seed), int(j), int(k), int(step), mean, sd))


class Network:
    """Element counts z [3, n] (float64: axon, excitatory and inhibitory dendrite),
    bound elements [3, n] (int32) and the synapse list, with the oracle's record and
    step."""

    def __init__(self, vac_axon, vac_exc, vac_inh, capacity: int):
        self.n = int(np.asarray(vac_axon).size)
        self.z = np.ascontiguousarray(np.stack([vac_axon, vac_exc, vac_inh]).astype(np.float64))
        self.bound = np.zeros((3, self.n), np.int32)
        self.src = np.zeros(max(capacity, 1), np.int32)
        self.tgt = np.zeros(max(capacity, 1), np.int32)
        self.type = np.zeros(max(capacity, 1), np.uint8)
        self.m = 0

    def record(self, syn_src, syn_tgt, syn_type) -> None:
        ns = np.ascontiguousarray(syn_src, dtype=np.int32)
        nt = np.ascontiguousarray(syn_tgt, dtype=np.int32)
        ny = np.ascontiguousarray(syn_type, dtype=np.uint8)
        if self.m + ns.size > self.src.size:
            raise ValueError("synapse capacity exceeded")
        lib().oracle_plasticity_record(self.n, self.m, ns.size, _p(ns), _p(nt), _p(ny),
                                       _p(self.src), _p(self.tgt), _p(self.type),
                                       _p(self.bound))
        self.m += ns.size

    def step(self, seed: int, step: int, params=None):
        """Returns the vacant elements (axon, exc, inh) for the next update."""
        p = dict(PLASTICITY, **(params or {}))
        vac = np.zeros((3, self.n), np.int32)
        self.m = int(lib().oracle_plasticity_step(
            self.n, self.m, p["nu"], p["eps"], p["eta"], int(p["steps"]), p["ca_mean"],
            p["ca_sd"], p["delete_frac"], int(seed), int(step), _p(self.z), _p(self.bound),
            _p(self.src), _p(self.tgt), _p(self.type), _p(vac)))
        return vac[0].copy(), vac[1].copy(), vac[2].copy()

    def synapses(self):
        return self.src[:self.m].copy(), self.tgt[:self.m].copy(), self.type[:self.m].copy()


# Electrical activity (Sec. II) with the firing-rate approximation (Sec. IV-B):
# Izhikevich's regular-spiking (excitatory) and fast-spiking (inhibitory) neurons,
# uniform background current, calcium as a running average of spikes, frequencies
# exchanged every `delta` steps.
ACTIVITY = dict(a_exc=0.02, b_exc=0.2, c_exc=-65.0, d_exc=8.0, a_inh=0.1, b_inh=0.2,
                c_inh=-65.0, d_inh=2.0, w_exc=2.0, w_inh=4.0, bg_mean=4.5, bg_width=9.0,
                ca_beta=0.001, ca_tau=10000.0, epoch=100)

_ACT_KEYS = ("a_exc", "b_exc", "c_exc", "d_exc", "a_inh", "b_inh", "c_inh", "d_inh", "w_exc",
             "w_inh", "bg_mean", "bg_width", "ca_beta")


class Activity:
    """Per-neuron state of the electrical activity: v, u, calcium (float64), the
    spikes of the last step (uint8), the spike count of the running epoch (int32) and
    the frequency of the previous epoch (float64)."""

    def __init__(self, neuron_type, params=None):
        self.type = np.ascontiguousarray(neuron_type, dtype=np.uint8)
        self.n = self.type.size
        self.p = dict(ACTIVITY, **(params or {}))
        inh = self.type != 0
        c = np.where(inh, self.p["c_inh"], self.p["c_exc"])
        b = np.where(inh, self.p["b_inh"], self.p["b_exc"])
        self.v = np.ascontiguousarray(c, dtype=np.float64)
        self.u = np.ascontiguousarray(b * c, dtype=np.float64)
        self.ca = np.zeros(self.n, np.float64)
        self.spk = np.zeros(self.n, np.uint8)
        self.count = np.zeros(self.n, np.int32)
        self.freq = np.zeros(self.n, np.float64)

    def run(self, syn_src, syn_tgt, syn_type, seed: int, t0: int, steps: int, approx: int = 0,
            rank=None, last_input: bool = False):
        """`steps` steps from global step t0. approx: 0 every spike is exchanged, 1 the
        synapses between different ranks use the frequency, 2 every synapse does.
        Returns the number of spikes (and the inputs [2, n] of the last step)."""
        src = np.ascontiguousarray(syn_src, dtype=np.int32)
        tgt = np.ascontiguousarray(syn_tgt, dtype=np.int32)
        sty = np.ascontiguousarray(syn_type, dtype=np.uint8)
        rk = None if rank is None else np.ascontiguousarray(rank, dtype=np.int32)
        pv = np.array([self.p[k] for k in _ACT_KEYS], dtype=np.float64)
        li = np.zeros((2, self.n), np.int32) if last_input else None
        total = lib().oracle_activity_run(
            self.n, _p(self.type), _p(rk), src.size, _p(src), _p(tgt), _p(sty), int(approx),
            _p(pv), 1.0 / self.p["ca_tau"], 1.0 / self.p["epoch"], int(self.p["epoch"]),
            int(seed), int(t0), int(steps), _p(self.v), _p(self.u), _p(self.ca), _p(self.spk),
            _p(self.count), _p(self.freq), _p(li))
        return (int(total), li) if last_input else int(total)
