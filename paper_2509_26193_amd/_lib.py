"""ctypes binding of libmsp (include/msp.h): argument marshalling only.

Tensors must be CUDA (HIP) tensors on the current device with the dtypes below;
every computation runs in libmsp's HIP kernels. If libmsp.so has not been built,
importing the functions raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "msp.h")

MSP_OK = 0
MSP_ERR_INVALID = -1
MSP_ERR_OOM = -2
MSP_ERR_HIP = -3
MSP_ERR_CAPACITY = -4
MSP_ERR_DEVICE = -5
MSP_ERR_UNIMPLEMENTED = -6
MSP_ERR_TOO_LARGE = -7
MSP_NOALLOC_MAX_NEURONS = 1 << 16


class MspError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_dbl = ctypes.c_double

class SearchDiag(ctypes.Structure):
    _fields_ = [("z0", _vp), ("levels", _vp), ("visits", _vp), ("opens", _vp),
                ("visits0", _vp), ("opens0", _vp), ("kernel_ms", ctypes.POINTER(ctypes.c_float)),
                ("wave_steps", _vp), ("branch_level", ctypes.c_int32),
                ("phase2_requests", _vp), ("parts_per_tile", ctypes.c_int32),
                ("entries0", _vp)]


class SimSpec(ctypes.Structure):
    _fields_ = [("tree", _vp), ("neuron_type", _vp), ("vac_axon", _vp), ("sigma_um", _dbl),
                ("seed", _u64), ("target_out", _vp), ("elem_offset_out", _vp),
                ("capacity_S", _i64)]


class PlasticityParams(ctypes.Structure):
    _fields_ = [("growth_rate", _dbl), ("target_calcium", _dbl), ("growth_onset", _dbl),
                ("calcium_mean", _dbl), ("calcium_sd", _dbl), ("delete_fraction", _dbl),
                ("steps_per_update", _i32)]


class CycleState(ctypes.Structure):
    _fields_ = [("z", _vp), ("bound", _vp), ("syn_src", _vp), ("syn_tgt", _vp),
                ("syn_type", _vp), ("m", _vp), ("vac_axon", _vp), ("vac_exc", _vp),
                ("vac_inh", _vp), ("step", _vp), ("status", _vp), ("searches", _vp),
                ("formed", _vp)]


class ActivityParams(ctypes.Structure):
    _fields_ = [("a_exc", _dbl), ("b_exc", _dbl), ("c_exc", _dbl), ("d_exc", _dbl),
                ("a_inh", _dbl), ("b_inh", _dbl), ("c_inh", _dbl), ("d_inh", _dbl),
                ("w_exc", _dbl), ("w_inh", _dbl), ("bg_mean", _dbl), ("bg_width", _dbl),
                ("ca_beta", _dbl), ("ca_tau", _dbl), ("epoch", _i32)]


_SIGS = {
    "msp_status_string": (ctypes.c_char_p, [_i32]),
    "msp_sync": (_i32, [_vp]),
    "msp_build_octree": (_i32, [_vp, _i64, _vp, _dbl, _i32, _vp, ctypes.POINTER(_vp)]),
    "msp_update_vacant_counts": (_i32, [_vp, _vp, _vp, _vp]),
    "msp_find_targets": (_i32, [_vp, _vp, _vp, _dbl, _dbl, _u64, _u64, _vp, _vp, _i64, _vp]),
    "msp_find_targets_noalloc": (_i32, [_vp, _vp, _vp, _dbl, _dbl, _u64, _u64, _vp, _vp, _i64,
                                        _vp]),
    "msp_find_targets_diag": (_i32, [_vp, _vp, _vp, _dbl, _dbl, _u64, _u64, _vp, _vp, _i64,
                                     ctypes.POINTER(SearchDiag), _vp]),
    "msp_commit_synapses": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _u64, _u64, _vp, _vp, _vp,
                                   _i64, _vp, _vp]),
    "msp_commit_synapses_ex": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _u64, _u64, _vp, _vp,
                                      _vp, _i64, _vp, _vp, _vp]),
    "msp_free_octree": (None, [_vp]),
    "msp_free_octree_async": (_i32, [_vp, _vp]),
    "msp_release_workspace": (_i32, [_i32]),
    "msp_search_offsets": (_i32, [_vp, _i64, _vp, ctypes.POINTER(_i64), _vp]),
    "msp_last_device_error": (_i32, [_vp]),
    "msp_octree_info": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "msp_octree_export_topology": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "msp_octree_export_aggregates": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "msp_batch_create": (_i32, [ctypes.POINTER(SimSpec), _i32, _i32, ctypes.POINTER(_vp)]),
    "msp_find_targets_batched": (_i32, [_vp, ctypes.POINTER(SimSpec), _dbl, _u64, _vp]),
    "msp_batch_status": (_i32, [_vp, _vp, ctypes.POINTER(_i32)]),
    "msp_batch_free": (None, [_vp]),
    "msp_attraction_fwd": (_i32, [_vp, _vp, _vp, _dbl, _dbl, _vp, _vp]),
    "msp_attraction_bwd": (_i32, [_vp, _vp, _vp, _dbl, _dbl, _vp, _vp, _vp, _vp]),
    "msp_plasticity_record": (_i32, [_i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _i64, _i64, _vp,
                                     _vp]),
    "msp_plasticity_step": (_i32, [_i64, ctypes.POINTER(PlasticityParams), _u64, _u64, _vp, _vp,
                                   _vp, _vp, _vp, _i64, ctypes.POINTER(_i64), _vp, _vp, _vp, _vp]),
    "msp_cycle_create": (_i32, [_vp, _vp, _dbl, _dbl, _u64, ctypes.POINTER(PlasticityParams),
                                _i64, _i64, ctypes.POINTER(CycleState), _i32,
                                ctypes.POINTER(_vp)]),
    "msp_cycle_run": (_i32, [_vp, _i32, _vp]),
    "msp_cycle_free": (None, [_vp]),
    "msp_activity_init": (_i32, [_i64, _vp, ctypes.POINTER(ActivityParams), _vp, _vp, _vp, _vp,
                                 _vp, _vp, _vp]),
    "msp_activity_run": (_i32, [_i64, _vp, _vp, _i64, _vp, _vp, _vp, _i32,
                                ctypes.POINTER(ActivityParams), _u64, _u64, _i32, _vp, _vp, _vp,
                                _vp, _vp, _vp, _vp, _vp, _vp]),
}

MSP_BATCH_GRAPH = 1
MSP_BATCH_AUTOTUNE = 2
MSP_CYCLE_GRAPH = 1
MSP_CYCLE_SEARCH_INVALID = 1
MSP_CYCLE_SEARCH_CAPACITY = 2
MSP_CYCLE_SYN_CAPACITY = 4
MSP_CYCLE_DEVICE = 8

_lib = None


def header_functions() -> list[str]:
    """Names of the functions declared in include/msp.h."""
    with open(HEADER) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(msp_[a-z0-9_]+)\s*\(", txt)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python paper_2509_26193_amd/build_lib.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(st: int) -> str:
    return lib().msp_status_string(int(st)).decode()


def _check(st: int, what: str) -> None:
    if st != MSP_OK:
        raise MspError(st, what)


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str, numel: int | None = None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


def _opt(t, dtype, name, numel=None):
    return None if t is None else _dev(t, dtype, name, numel)


class Octree:
    """Handle of an octree built by msp_build_octree (owned by libmsp)."""

    def __init__(self, handle: int, n: int, device: torch.device):
        self._h = handle
        self.n = n
        self.device = device

    @property
    def handle(self) -> int:
        if not self._h:
            raise ValueError("octree was freed")
        return self._h

    @property
    def num_nodes(self) -> int:
        nn = _i64()
        nN = _i64()
        _check(lib().msp_octree_info(self.handle, ctypes.byref(nn), ctypes.byref(nN)), "octree_info")
        return int(nN.value)

    def free(self, stream=None) -> None:
        """Stream-ordered release: the memory returns to the library's pool after the
        work queued so far on `stream` (default: the current stream). Uses of the
        octree on other streams must be ordered before that point by the caller."""
        if self._h:
            h, self._h = self._h, None
            _check(lib().msp_free_octree_async(h, _stream(stream)), "free_octree")

    def __del__(self):
        # at collection time the caller's stream order is unknown: wait for the device
        try:
            if self._h:
                h, self._h = self._h, None
                lib().msp_free_octree(h)
        except Exception:
            pass

    def last_device_error(self) -> int:
        return int(lib().msp_last_device_error(self.handle))

    def export_topology(self, stream=None) -> dict:
        N = self.num_nodes
        dev = self.device
        out = dict(order=torch.empty(self.n, dtype=torch.int32, device=dev),
                   keys=torch.empty(self.n, dtype=torch.int64, device=dev),
                   depth=torch.empty(N, dtype=torch.int32, device=dev),
                   begin=torch.empty(N, dtype=torch.int64, device=dev),
                   end=torch.empty(N, dtype=torch.int64, device=dev),
                   subtree_end=torch.empty(N, dtype=torch.int64, device=dev))
        _check(lib().msp_octree_export_topology(
            self.handle, out["order"].data_ptr(), out["keys"].data_ptr(), out["depth"].data_ptr(),
            out["begin"].data_ptr(), out["end"].data_ptr(), out["subtree_end"].data_ptr(),
            _stream(stream)), "export_topology")
        return out

    def export_aggregates(self, type_: int, stream=None):
        N = self.num_nodes
        v = torch.empty(N, dtype=torch.int64, device=self.device)
        c = torch.empty((N, 3), dtype=torch.float64, device=self.device)
        _check(lib().msp_octree_export_aggregates(self.handle, int(type_), v.data_ptr(),
                                                  c.data_ptr(), _stream(stream)),
               "export_aggregates")
        return v, c


def build_octree(pos: torch.Tensor, box_min, box_edge: float, leaf_size: int = 1,
                 stream=None) -> Octree:
    n = pos.shape[0]
    p = _dev(pos, torch.float64, "pos", 3 * n)
    bm = (ctypes.c_double * 3)(*[float(x) for x in box_min])
    h = _vp()
    _check(lib().msp_build_octree(p, n, bm, float(box_edge), int(leaf_size), _stream(stream),
                                  ctypes.byref(h)), "build_octree")
    return Octree(h.value, n, pos.device)


def search_offsets(vac_axon: torch.Tensor, elem_offset_out: torch.Tensor | None = None,
                   stream=None):
    """(elem_offset[n+1], S): the CSR offsets of the searches (exclusive prefix sum of
    vac_axon) and their number, computed by the library (waits on the stream)."""
    n = vac_axon.numel()
    if elem_offset_out is None:
        elem_offset_out = torch.empty(n + 1, dtype=torch.int64, device=vac_axon.device)
    S = _i64(0)
    _check(lib().msp_search_offsets(_dev(vac_axon, torch.int32, "vac_axon", n), n,
                                    _dev(elem_offset_out, torch.int64, "elem_offset_out", n + 1),
                                    ctypes.byref(S), _stream(stream)), "search_offsets")
    return elem_offset_out, int(S.value)


def release_workspace(device=None) -> None:
    """Free the search working memory the library keeps on `device` (default: the
    current device); the next search allocates it again."""
    d = torch.cuda.current_device() if device is None else torch.device(device).index
    _check(lib().msp_release_workspace(int(d if d is not None else 0)), "release_workspace")


def update_vacant_counts(tree: Octree, vac_exc: torch.Tensor, vac_inh: torch.Tensor,
                         stream=None) -> None:
    _check(lib().msp_update_vacant_counts(tree.handle, _dev(vac_exc, torch.int32, "vac_exc", tree.n),
                                          _dev(vac_inh, torch.int32, "vac_inh", tree.n),
                                          _stream(stream)), "update_vacant_counts")


def find_targets(tree: Octree, neuron_type: torch.Tensor, vac_axon: torch.Tensor, sigma: float,
                 theta: float, seed: int, step: int, target_out: torch.Tensor | None = None,
                 elem_offset_out: torch.Tensor | None = None, diag: bool = False,
                 counters: bool = False, timing: dict | None = None, stream=None,
                 branch_level: int = 0, phase2: dict | None = None, parts: int = 0):
    """Returns (target[S], elem_offset[n+1]); with diag also (z0[S], levels[S]); with
    counters also a dict of visits/opens/visits0/opens0/entries0 [S] and wave_steps. target_out may be a
    preallocated int32 buffer of any capacity >= S. If `timing` is a dict, the kernel
    durations (HIP events on the launch stream) are stored under "sweep_ms" (level-0
    sweep), "draw_ms" (draws and restarts, both phases), "phase2_ms" (the second phase)
    and "kernel_ms" (all). branch_level selects the two-phase search (restarts from
    cells at that depth or deeper run in a second pass, in cell order; 0: the library's
    default); if `phase2` is a dict, phase2["requests"] is set to the number of
    second-phase requests. parts: the level-0 walk of every tile in 1, 2, 4 or 8
    pre-order parts (0: the library's choice)."""
    n = tree.n
    dev = tree.device
    ty = _dev(neuron_type, torch.uint8, "neuron_type", n)
    a = _dev(vac_axon, torch.int32, "vac_axon", n)
    if elem_offset_out is None:
        elem_offset_out = torch.empty(n + 1, dtype=torch.int64, device=dev)
    off = _dev(elem_offset_out, torch.int64, "elem_offset_out", n + 1)
    st = _stream(stream)
    ms = (ctypes.c_float * 3)(0.0, 0.0, 0.0)
    extra = {}
    if target_out is None:                  # size the output once instead of retrying
        _, S0 = search_offsets(vac_axon, elem_offset_out, stream)
        target_out = torch.empty(max(S0, 1), dtype=torch.int32, device=dev)
    for attempt in range(2):
        cap = 0 if target_out is None else target_out.numel()
        d = SearchDiag()
        if diag:
            extra["z0"] = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
            extra["levels"] = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        if counters:
            for k in ("visits", "opens", "visits0", "opens0", "entries0"):
                extra[k] = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
            extra["wave_steps"] = torch.zeros(1, dtype=torch.int64, device=dev)
        for k, v in extra.items():
            setattr(d, k, v.data_ptr())
        d.branch_level = int(branch_level)
        d.parts_per_tile = int(parts)
        if phase2 is not None:
            nreq = torch.zeros(1, dtype=torch.int64, device=dev)
            d.phase2_requests = nreq.data_ptr()
        if timing is not None:
            d.kernel_ms = ctypes.cast(ms, ctypes.POINTER(ctypes.c_float))
        tp = None if target_out is None else _dev(target_out, torch.int32, "target_out")
        rc = lib().msp_find_targets_diag(tree.handle, ty, a, float(sigma), float(theta), int(seed),
                                         int(step), tp, off, cap, ctypes.byref(d), st)
        if rc == MSP_ERR_CAPACITY and attempt == 0:
            S = int(elem_offset_out[n].item())
            target_out = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
            continue
        _check(rc, "find_targets")
        break
    S = int(elem_offset_out[n].item())
    if target_out is None:
        target_out = torch.empty(0, dtype=torch.int32, device=dev)
    if timing is not None:
        timing["sweep_ms"] = float(ms[0])
        timing["draw_ms"] = float(ms[1]) + float(ms[2])
        timing["phase2_ms"] = float(ms[2])
        timing["kernel_ms"] = float(ms[0]) + float(ms[1]) + float(ms[2])
    if phase2 is not None:
        phase2["requests"] = int(nreq.item())
    out = [target_out[:S], elem_offset_out]
    if diag:
        out += [extra["z0"][:S], extra["levels"][:S]]
    if counters:
        c = {k: extra[k][:S] for k in ("visits", "opens", "visits0", "opens0", "entries0")}
        c["wave_steps"] = extra["wave_steps"]
        out.append(c)
    return tuple(out)


def commit_synapses(target: torch.Tensor, elem_offset: torch.Tensor, neuron_type: torch.Tensor,
                    vac_axon: torch.Tensor, vac_exc: torch.Tensor, vac_inh: torch.Tensor,
                    seed: int, step: int, syn_capacity: int | None = None,
                    return_accepted: bool = False, stream=None) -> dict:
    """Accept/decline all requests; vac_* are updated in place. Returns the synapses."""
    n = vac_axon.numel()
    dev = vac_axon.device
    S = int(elem_offset[n].item()) if syn_capacity is None else None
    cap = S if syn_capacity is None else int(syn_capacity)
    src = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    tgt = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    sty = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
    nf = torch.zeros(1, dtype=torch.int64, device=dev)
    Sx = target.numel()
    acc = torch.empty(max(Sx, 1), dtype=torch.uint8, device=dev) if return_accepted else None
    tp = _dev(target, torch.int32, "target") if target.numel() > 0 else None
    rc = lib().msp_commit_synapses_ex(tp, _dev(elem_offset, torch.int64, "elem_offset", n + 1),
                                      _dev(neuron_type, torch.uint8, "neuron_type", n), n,
                                      _dev(vac_axon, torch.int32, "vac_axon", n),
                                      _dev(vac_exc, torch.int32, "vac_exc", n),
                                      _dev(vac_inh, torch.int32, "vac_inh", n), int(seed), int(step),
                                      src.data_ptr(), tgt.data_ptr(), sty.data_ptr(), cap,
                                      nf.data_ptr(), None if acc is None else acc.data_ptr(),
                                      _stream(stream))
    _check(rc, "commit_synapses")
    m = int(nf.item())
    out = dict(syn_src=src[:m], syn_tgt=tgt[:m], syn_type=sty[:m], n_formed=m)
    if return_accepted:
        out["accepted"] = acc[:Sx]
    return out


def sync(stream=None) -> None:
    _check(lib().msp_sync(_stream(stream)), "sync")


class Batch:
    """A plan for searching many independent simulations with one set of launches.

    sims: list of dicts with keys tree (Octree), neuron_type (uint8), vac_axon (int32),
    sigma (float), seed (int), and optionally target_out (int32, capacity >= searches)
    and elem_offset_out (int64, n + 1). Missing outputs are allocated from the
    searches implied by vac_axon. Per simulation the targets equal find_targets'."""

    def __init__(self, sims, graph: bool = False, autotune: bool = False):
        self._h = None
        self.n_sims = len(sims)
        self.sims = [dict(s) for s in sims]
        for d in self.sims:
            n = d["tree"].n
            dev = d["tree"].device
            if d.get("elem_offset_out") is None:
                d["elem_offset_out"] = torch.empty(n + 1, dtype=torch.int64, device=dev)
            if d.get("target_out") is None:
                _, S = search_offsets(d["vac_axon"], d["elem_offset_out"])
                d["target_out"] = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
        arr = self._specs()
        flags = (MSP_BATCH_GRAPH if graph else 0) | (MSP_BATCH_AUTOTUNE if autotune else 0)
        h = _vp()
        _check(lib().msp_batch_create(arr, self.n_sims, flags, ctypes.byref(h)), "batch_create")
        self._h = h.value

    def _specs(self):
        arr = (SimSpec * self.n_sims)()
        for k, d in enumerate(self.sims):
            n = d["tree"].n
            arr[k].tree = d["tree"].handle
            arr[k].neuron_type = _dev(d["neuron_type"], torch.uint8, "neuron_type", n)
            arr[k].vac_axon = _dev(d["vac_axon"], torch.int32, "vac_axon", n)
            arr[k].sigma_um = float(d["sigma"])
            arr[k].seed = int(d["seed"])
            arr[k].target_out = _dev(d["target_out"], torch.int32, "target_out")
            arr[k].elem_offset_out = _dev(d["elem_offset_out"], torch.int64, "elem_offset_out", n + 1)
            arr[k].capacity_S = d["target_out"].numel()
        return arr

    def run(self, theta: float, step: int, update: bool = False, stream=None) -> None:
        """Queue one batched search (asynchronous). With update=True the current
        buffers and parameters in self.sims are re-sent."""
        arr = self._specs() if update else None
        _check(lib().msp_find_targets_batched(self._h, arr, float(theta), int(step),
                                              _stream(stream)), "find_targets_batched")

    def status(self, stream=None) -> list:
        st = (_i32 * self.n_sims)()
        lib().msp_batch_status(self._h, _stream(stream), st)
        return [int(x) for x in st]

    def results(self, k: int):
        """(target[S], elem_offset[n+1]) of simulation k after a run."""
        d = self.sims[k]
        off = d["elem_offset_out"]
        S = int(off[-1].item())
        return d["target_out"][:S], off

    def free(self) -> None:
        if self._h:
            lib().msp_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def attraction_fwd(tree: Octree, neuron_type, vac_axon, sigma: float, theta: float,
                   stream=None) -> torch.Tensor:
    """Z[n] (float32): level-0 normaliser of every neuron with vacant axonal elements."""
    n = tree.n
    Z = torch.empty(n, dtype=torch.float32, device=tree.device)
    _check(lib().msp_attraction_fwd(tree.handle, _dev(neuron_type, torch.uint8, "neuron_type", n),
                                    _dev(vac_axon, torch.int32, "vac_axon", n), float(sigma),
                                    float(theta), Z.data_ptr(), _stream(stream)), "attraction_fwd")
    return Z


def attraction_bwd(tree: Octree, neuron_type, vac_axon, sigma: float, theta: float,
                   gZ: torch.Tensor, stream=None):
    """(dpos[n][3] float32, dsigma float64 0-d tensor) for upstream gradient gZ[n]."""
    n = tree.n
    dpos = torch.empty((n, 3), dtype=torch.float32, device=tree.device)
    ds = torch.empty((), dtype=torch.float64, device=tree.device)
    g = gZ.to(torch.float32).contiguous()
    _check(lib().msp_attraction_bwd(tree.handle, _dev(neuron_type, torch.uint8, "neuron_type", n),
                                    _dev(vac_axon, torch.int32, "vac_axon", n), float(sigma),
                                    float(theta), _dev(g, torch.float32, "gZ", n), dpos.data_ptr(),
                                    ds.data_ptr(), _stream(stream)), "attraction_bwd")
    return dpos, ds


class AttractionFn(torch.autograd.Function):
    """Z = expected attraction of each axon-bearing neuron, differentiable in the
    positions and in sigma (acceptance decisions held fixed). The octree must have
    been built from `pos` and refreshed with the current dendritic vacancies."""

    @staticmethod
    def forward(ctx, pos, sigma, tree, neuron_type, vac_axon, theta):
        s = float(sigma.detach())
        Z = attraction_fwd(tree, neuron_type, vac_axon, s, theta)
        ctx.tree = tree
        ctx.args = (neuron_type, vac_axon, s, theta)
        ctx.sigma_dtype = sigma.dtype
        return Z

    @staticmethod
    def backward(ctx, gZ):
        neuron_type, vac_axon, s, theta = ctx.args
        dpos, ds = attraction_bwd(ctx.tree, neuron_type, vac_axon, s, theta, gZ)
        return dpos.to(torch.float64), ds.to(ctx.sigma_dtype), None, None, None, None


def attraction(pos: torch.Tensor, sigma: torch.Tensor, tree: Octree, neuron_type, vac_axon,
               theta: float) -> torch.Tensor:
    """Differentiable Z (see AttractionFn)."""
    return AttractionFn.apply(pos, sigma, tree, neuron_type, vac_axon, theta)


PLASTICITY = dict(growth_rate=0.001, target_calcium=0.7, growth_onset=0.4, calcium_mean=0.7,
                  calcium_sd=0.1, delete_fraction=0.1, steps_per_update=100)


class Network:
    """Device state of the plasticity between updates: element counts z [3][n]
    (float64; kinds axon, excitatory dendrite, inhibitory dendrite), bound elements
    [3][n] (int32) and the synapse list (capacity entries, m used)."""

    def __init__(self, vac_axon: torch.Tensor, vac_exc: torch.Tensor, vac_inh: torch.Tensor,
                 capacity: int):
        dev = vac_axon.device
        self.n = vac_axon.numel()
        self.z = torch.stack([vac_axon, vac_exc, vac_inh]).to(torch.float64).contiguous()
        self.bound = torch.zeros((3, self.n), dtype=torch.int32, device=dev)
        self.src = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        self.tgt = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        self.type = torch.empty(max(capacity, 1), dtype=torch.uint8, device=dev)
        self.m = 0

    def record(self, syn_src: torch.Tensor, syn_tgt: torch.Tensor, syn_type: torch.Tensor,
               stream=None) -> None:
        """Append synapses (e.g. commit_synapses' output) and bind their elements."""
        k = syn_src.numel()
        if k == 0:
            return
        _check(lib().msp_plasticity_record(
            self.n, _dev(syn_src, torch.int32, "syn_src", k), _dev(syn_tgt, torch.int32, "syn_tgt", k),
            _dev(syn_type, torch.uint8, "syn_type", k), k, self.src.data_ptr(),
            self.tgt.data_ptr(), self.type.data_ptr(), self.m, self.src.numel(),
            self.bound.data_ptr(), _stream(stream)), "plasticity_record")
        self.m += k

    def step(self, seed: int, step: int, params: dict | None = None, stream=None):
        """Growth, deletion and retraction after update `step`; returns the vacant
        elements (axon, exc, inh) as int32 device tensors for the next update."""
        p = PlasticityParams(**dict(PLASTICITY, **(params or {})))
        va = torch.empty(self.n, dtype=torch.int32, device=self.z.device)
        ve = torch.empty_like(va)
        vi = torch.empty_like(va)
        m_out = _i64(0)
        _check(lib().msp_plasticity_step(
            self.n, ctypes.byref(p), int(seed), int(step), self.z.data_ptr(), self.bound.data_ptr(),
            self.src.data_ptr(), self.tgt.data_ptr(), self.type.data_ptr(), self.m,
            ctypes.byref(m_out), va.data_ptr(), ve.data_ptr(), vi.data_ptr(), _stream(stream)),
            "plasticity_step")
        self.m = int(m_out.value)
        return va, ve, vi

    def synapses(self):
        return self.src[:self.m], self.tgt[:self.m], self.type[:self.m]


class Cycle:
    """Update cycles of a Network on a fixed octree (msp_cycle_*): each update refreshes
    the octree's vacancies, searches, commits, records and runs the plasticity step,
    exactly as the separate calls do, with every count on the device and no host wait;
    graph=True replays one captured update. The cycle takes over the network's
    synapse count and the vacancy tensors (updated in place); `step` is the first
    update's step."""

    def __init__(self, tree: Octree, neuron_type: torch.Tensor, net: "Network",
                 vac_axon: torch.Tensor, vac_exc: torch.Tensor, vac_inh: torch.Tensor,
                 sigma_um: float, theta: float, seed: int, step: int = 0,
                 params: dict | None = None, search_capacity: int | None = None,
                 graph: bool = True):
        n = net.n
        dev = net.z.device
        self.net = net
        for t, name in ((vac_axon, "vac_axon"), (vac_exc, "vac_exc"), (vac_inh, "vac_inh")):
            _dev(t, torch.int32, name, n)
        self.va, self.ve, self.vi = vac_axon, vac_exc, vac_inh
        # device scalars: m, step, searches, formed (int64) and the status word
        self.i64 = torch.tensor([net.m, int(step), 0, 0], dtype=torch.int64, device=dev)
        self.status_word = torch.zeros(1, dtype=torch.int32, device=dev)
        p = PlasticityParams(**dict(PLASTICITY, **(params or {})))
        ptr = self.i64.data_ptr()
        self._state = CycleState(net.z.data_ptr(), net.bound.data_ptr(), net.src.data_ptr(),
                                 net.tgt.data_ptr(), net.type.data_ptr(), ptr,
                                 self.va.data_ptr(), self.ve.data_ptr(), self.vi.data_ptr(),
                                 ptr + 8, self.status_word.data_ptr(), ptr + 16, ptr + 24)
        cap = int(search_capacity) if search_capacity else max(1, 3 * n)
        _dev(neuron_type, torch.uint8, "neuron_type", n)
        self._type = neuron_type
        self._tree = tree
        h = _vp()
        _check(lib().msp_cycle_create(tree.handle, neuron_type.data_ptr(), float(sigma_um),
                                      float(theta), int(seed), ctypes.byref(p), cap,
                                      net.src.numel(), ctypes.byref(self._state),
                                      MSP_CYCLE_GRAPH if graph else 0, ctypes.byref(h)),
               "cycle_create")
        self.handle = h.value

    def run(self, updates: int = 1, stream=None) -> None:
        """Enqueue `updates` updates (no host wait)."""
        _check(lib().msp_cycle_run(self.handle, int(updates), _stream(stream)), "cycle_run")

    def va_ve_vi(self):
        """The vacancy tensors the cycle reads and rewrites (axon, exc, inh)."""
        return self.va, self.ve, self.vi

    def status(self) -> int:
        """The OR of the status bits of the updates run so far (waits for them)."""
        return int(self.status_word.item())

    def counts(self) -> dict:
        """m, the next step, and the last update's searches and synapses formed (waits);
        also sets the network's host-side synapse count."""
        m, step, searches, formed = (int(v) for v in self.i64.cpu())
        self.net.m = m
        return dict(m=m, step=step, searches=searches, formed=formed)

    def free(self) -> None:
        if self.handle:
            lib().msp_cycle_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


ACTIVITY = dict(a_exc=0.02, b_exc=0.2, c_exc=-65.0, d_exc=8.0, a_inh=0.1, b_inh=0.2,
                c_inh=-65.0, d_inh=2.0, w_exc=2.0, w_inh=4.0, bg_mean=4.5, bg_width=9.0,
                ca_beta=0.001, ca_tau=10000.0, epoch=100)


class Activity:
    """Device state of the electrical activity (msp_activity_run): v, u, calcium and
    the previous epoch's frequency (float64), the last step's spikes (uint8) and the
    running epoch's spike count (int32), for neurons of the given types."""

    def __init__(self, neuron_type: torch.Tensor, params: dict | None = None):
        self.type = neuron_type
        self.n = neuron_type.numel()
        self.p = dict(ACTIVITY, **(params or {}))
        dev = neuron_type.device
        f64 = dict(dtype=torch.float64, device=dev)
        self.v = torch.empty(self.n, **f64)
        self.u = torch.empty(self.n, **f64)
        self.calcium = torch.empty(self.n, **f64)
        self.spiked = torch.empty(self.n, dtype=torch.uint8, device=dev)
        self.count = torch.empty(self.n, dtype=torch.int32, device=dev)
        self.freq = torch.empty(self.n, **f64)
        P = ActivityParams(*[self.p[f] for f, _ in ActivityParams._fields_])
        _check(lib().msp_activity_init(
            self.n, _dev(self.type, torch.uint8, "neuron_type", self.n), ctypes.byref(P),
            self.v.data_ptr(), self.u.data_ptr(), self.calcium.data_ptr(), self.spiked.data_ptr(),
            self.count.data_ptr(), self.freq.data_ptr(), _stream(None)), "activity_init")

    def run(self, syn_src: torch.Tensor, syn_tgt: torch.Tensor, syn_type: torch.Tensor,
            seed: int, t0: int, steps: int, approx: int = 0, rank: torch.Tensor | None = None,
            last_input: bool = False, spikes: torch.Tensor | None = None, stream=None):
        """Steps t0 .. t0 + steps - 1. approx: 0 exchange every spike, 1 use the
        frequency on synapses between different ranks, 2 on every synapse. Returns the
        inputs [2, n] of the last step when last_input is set. `spikes` (device int64
        [1]) is incremented by the number of spikes."""
        m = syn_src.numel()
        li = torch.empty((2, self.n), dtype=torch.int32, device=self.type.device) \
            if last_input else None
        P = ActivityParams(*[self.p[f] for f, _ in ActivityParams._fields_])
        _check(lib().msp_activity_run(
            self.n, _dev(self.type, torch.uint8, "neuron_type", self.n),
            None if rank is None else _dev(rank, torch.int32, "rank", self.n), m,
            _dev(syn_src, torch.int32, "syn_src", m) if m else None,
            _dev(syn_tgt, torch.int32, "syn_tgt", m) if m else None,
            _dev(syn_type, torch.uint8, "syn_type", m) if m else None, int(approx),
            ctypes.byref(P), int(seed), int(t0), int(steps), self.v.data_ptr(),
            self.u.data_ptr(), self.calcium.data_ptr(), self.spiked.data_ptr(),
            self.count.data_ptr(), self.freq.data_ptr(),
            None if li is None else li.data_ptr(),
            None if spikes is None else _dev(spikes, torch.int64, "spikes", 1),
            _stream(stream)), "activity_run")
        return li
