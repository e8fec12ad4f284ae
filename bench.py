#!/usr/bin/env python3
"""Throughput of the MSP connectivity update (arXiv 2509.26193) on one MI355X.

One step = one whole connectivity update over the resident synthetic brain:
build the octree, refresh the vacancy aggregates, run the Barnes-Hut target search for
every vacant axonal element, commit the accepted synapses. The counts are restored
from a resident copy at the start of each step so that every step does the same work.

Prints one JSON line (rank 0). Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # MI355X HBM3E, bytes/s
EXP2_PEAK = 256 * 64 * 2.4e9 / 4   # float32 exp2 per second, quarter-rate transcendental
FP64_VECTOR_PEAK = 78.6e12  # MI355X fp64 vector FLOP/s (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
# vector lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, every
# vector operation (an FMA included) counted once (= the fp64 vector peak / 2)
VALU_OPS_PEAK = 256 * 4 * 16 * 2.4e9
REC_BYTES = 16             # one per-type node record {x, y, z, count} at 4 bytes each
OPEN_BYTES = 8             # child link + mask + depth of an opened node
SRC_BYTES = 16             # source record
OUT_BYTES = 4              # one int32 target
# vector operations the method needs per source and level-0 record (the per-visit
# operation model): a record with vacancy 8 (3 differences and 3 multiply-adds for
# d^2, the theta^2 d^2 product and its compare), an accepted entry 3 more (exp2, the
# product with v, the running sum), a record without vacancy 1 (the zero test)
OPS_VISIT, OPS_ENTRY, OPS_EMPTY = 8, 3, 1
WALK_REC_BYTES = 32        # the 32-byte record one wave step of the shared walk loads
WALK_SRC_BYTES = 40        # per source: position 24 B, leaf 4 B, worklist 4 B, Z out 8 B
PAPER_CONTEXT = dict(
    value=0.93e6, unit="searches/s",
    hardware="1024 MPI ranks on Lichtenberg 2 nodes (2x Intel Xeon Platinum 8470Q, 52 cores "
             "each, 2.1 GHz; InfiniBand HDR100)",
    workload="1024 x 65,536 neurons, theta 0.2, 10 connectivity updates",
    note="derived, not printed: at least 67.1 M searches (one per neuron on the first "
         "update) in the 72 s of Barnes-Hut computation (Sec. V-B, V-E); another workload "
         "and machine, context only (vs_baseline stays null)")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name, theta):
    from synth_inputs import config_clusters, config_large, config_small
    if name == "large":
        w = config_large()
    elif name == "clusters":
        w = config_clusters(theta=0.3 if theta is None else theta)
    elif name == "small":
        w = config_small()
    else:
        raise SystemExit(f"unknown workload {name}")
    if theta is not None:
        w.theta = float(theta)
    return w


def algorithmic_bytes(cnt, off):
    """Bytes the method must read for one launch: each source's level-0 list once
    (records visited, nodes opened, the source), each search's restart lists, and
    one output per search."""
    v = cnt["visits"].astype(np.int64)
    o = cnt["opens"].astype(np.int64)
    v0 = cnt["visits0"].astype(np.int64)
    o0 = cnt["opens0"].astype(np.int64)
    first = off[:-1][np.diff(off) > 0]          # first element of every source
    lvl0 = (REC_BYTES * v0[first] + OPEN_BYTES * o0[first] + SRC_BYTES).sum()
    rest = (REC_BYTES * (v - v0) + OPEN_BYTES * (o - o0) + OUT_BYTES).sum()
    return int(lvl0 + rest), int(v0[first].sum() + (v - v0).sum())


def sweep_bytes(cnt, off):
    """Algorithmic bytes of the level-0 sweep kernel: every source's level-0 records
    visited, nodes opened and the source record, once per source."""
    v0 = cnt["visits0"].astype(np.int64)
    o0 = cnt["opens0"].astype(np.int64)
    first = off[:-1][np.diff(off) > 0]
    return int((REC_BYTES * v0[first] + OPEN_BYTES * o0[first] + SRC_BYTES).sum())


def sweep_alu_ops(cnt, off):
    """Vector operations the method needs in the level-0 sweep, from the exact
    per-search counters of one counting launch (first element of every source)."""
    first = off[:-1][np.diff(off) > 0]
    v0 = cnt["visits0"][first].astype(np.int64)
    o0 = cnt["opens0"][first].astype(np.int64)
    e0 = cnt["entries0"][first].astype(np.int64)
    empty = np.maximum(v0 - o0 - e0, 0)
    return int((OPS_VISIT * (v0 - empty) + OPS_ENTRY * e0 + OPS_EMPTY * empty).sum())


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_counters(workload):
    """Issue counters of the sweep from the committed rocprofv3 summary, if they were
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "search_sweep_counters.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(workload)
    if not e or e.get("kernel_sources") != kernel_sources_hash():
        return None
    return e


def oracle_threads():
    """Host threads the oracle runs on: every core, at most 64."""
    return min(os.cpu_count() or 1, 64)


def counted(msp, tree, ty, va, sigma, theta, seed, step):
    """Per-search visit/open counters of one counting launch, on the host."""
    _, off, _, _, cnt = msp.find_targets(tree, ty, va, sigma, theta, seed, step, diag=True,
                                         counters=True)
    h = {k: v.cpu().numpy() for k, v in cnt.items() if k != "wave_steps"}
    return h, off.cpu().numpy()


def hbm_roofline(bytes_, seconds, what):
    return dict(bound="hbm", unit="GB/s", achieved=bytes_ / seconds / 1e9,
                peak=HBM_PEAK / 1e9, frac=bytes_ / seconds / HBM_PEAK, bytes=int(bytes_),
                basis=what)


def alu_roofline(ops, logical_bytes, seconds, what):
    """The search rows' bound: vector operations the method needs over the kernels'
    time against the vector-op peak; the logical traversal bytes beside it
    (every lane charged separately, so above 1 where lanes share record loads)."""
    return dict(bound="alu", unit="Tops/s", achieved=ops / seconds / 1e12,
                peak=VALU_OPS_PEAK / 1e12, frac=ops / seconds / VALU_OPS_PEAK, ops=int(ops),
                basis=what, logical_bytes=int(logical_bytes),
                logical_traversal_frac=logical_bytes / seconds / HBM_PEAK)


def kernel_sources_hash():
    """Hash of the search kernel sources with comments and whitespace removed: measured
    HBM traffic is reported only for the kernel code it was measured on."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("search.hpp", "search_wave.hpp", "batch.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2509_26193_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per sweep launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "search_sweep_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    e = d.get(workload)
    if not e or e.get("kernel_sources") != kernel_sources_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def copy_calibration():
    """A plain device copy of known size (1 GiB read + 1 GiB written per launch), run
    under the same rocprofv3 counters to scale FETCH_SIZE / WRITE_SIZE."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: 3 launches of a 1 GiB device-to-device copy")


def cpu_baseline(w, gpu_target, sample, threads):
    from oracle import oracle as orc
    t0 = time.time()
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    tb = time.time() - t0
    t0 = time.time()
    t.update_counts(w.vac_exc, w.vac_inh)
    tr = time.time() - t0
    off, src, elem = orc.search_list(w.vac_axon)
    rng = np.random.default_rng(1234)
    m = min(sample, src.size)
    q = np.sort(rng.choice(src.size, size=m, replace=False))
    log(f"oracle tree built in {tb:.1f} s, refreshed in {tr:.1f} s; timing {m} searches")
    t0 = time.time()
    r = t.find_targets(w.neuron_type, w.sigma, w.theta, w.seed, w.step, src[q], elem[q],
                       nthreads=threads)
    ts = time.time() - t0
    differ = int((r["target"] != gpu_target[q]).sum())
    outside = int(((r["target"] != gpu_target[q]) & ~(r["window"] < 1e-6)).sum())
    window_hits = int((r["window"] < 1e-6).sum())
    # the same oracle on one thread, on the first 5000 of those searches
    q1 = q[:5000]
    t0 = time.time()
    t.find_targets(w.neuron_type, w.sigma, w.theta, w.seed, w.step, src[q1], elem[q1], nthreads=1)
    t1 = time.time() - t0
    return dict(value=m / ts, unit="searches/s", cores=threads, kind="oracle",
                sample=(f"{m} random searches of the {src.size} in one update of {w.name} "
                        f"(fp64 oracle, OpenMP {threads} threads); tree build {tb:.1f} s and "
                        f"refresh {tr:.1f} s not included"),
                cpu_model=cpu_model(), nproc=os.cpu_count(),
                one_thread=dict(value=q1.size / t1, unit="searches/s",
                                sample=f"the first {q1.size} of those searches, 1 thread"),
                parity=dict(targets="the last timed step's", sampled=m, differing=differ,
                            differing_share=differ / max(m, 1), share_bound=1e-4,
                            outside_window=outside, oracle_window_hits=window_hits))


def bench_plain_update(msp, torch, w, steps, warmup):
    """Whole-update throughput (build + refresh + search + commit) of one workload."""
    dev = torch.device("cuda:0")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    pos = T(w.pos, torch.float64)
    ty = T(w.neuron_type, torch.uint8)
    va0, ve0, vi0 = T(w.vac_axon, torch.int32), T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32)
    va, ve, vi = va0.clone(), ve0.clone(), vi0.clone()
    S = w.searches
    tgt_buf = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
    kern = []

    def step():
        tree = msp.build_octree(pos, w.box_min, w.box_edge)
        va.copy_(va0); ve.copy_(ve0); vi.copy_(vi0)
        msp.update_vacant_counts(tree, ve, vi)
        tm = {}
        tgt, off = msp.find_targets(tree, ty, va, w.sigma, w.theta, w.seed, w.step,
                                    target_out=tgt_buf, timing=tm)
        msp.commit_synapses(tgt, off, ty, va, ve, vi, w.seed, w.step, syn_capacity=S)
        tree.free()
        kern.append(tm["kernel_ms"])

    for _ in range(warmup):
        step()
    kern.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    tree = msp.build_octree(pos, w.box_min, w.box_edge)
    msp.update_vacant_counts(tree, ve0, vi0)
    cnt, off = counted(msp, tree, ty, va0, w.sigma, w.theta, w.seed, w.step)
    tree.free()
    B, _ = algorithmic_bytes(cnt, off)
    ops = sweep_alu_ops(cnt, off)
    ks = float(np.mean(kern)) / 1e3
    # the oracle on 20000 sampled searches of the same update
    from oracle import oracle as orc
    t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
    t.update_counts(w.vac_exc, w.vac_inh)
    _, src, elem = orc.search_list(w.vac_axon)
    q = np.sort(np.random.default_rng(99).choice(src.size, size=min(20000, src.size),
                                                 replace=False))
    t0 = time.perf_counter()
    t.find_targets(w.neuron_type, w.sigma, w.theta, w.seed, w.step, src[q], elem[q],
                   nthreads=oracle_threads())
    t_or = time.perf_counter() - t0
    return dict(workload=w.name, neurons=w.n, searches=S, theta=w.theta, ms_per_update=sec * 1e3,
                searches_per_s=S / sec, search_kernels_ms=ks * 1e3,
                roofline=alu_roofline(ops, B, ks, "level-0 vector operations of the method / "
                                      "the search kernels' (sweep + draw) HIP-event time"),
                oracle=dict(value=q.size / t_or, unit="searches/s", cores=oracle_threads(),
                            kind="oracle", sample=f"{q.size} sampled searches of the same "
                            "update, tree build and refresh not included"))


def bench_two_phase(msp, torch, w, alg_bytes, alg_ops, branch_level=6, reps=4):
    """The two-phase (location-aware) search of Sec. IV-A on the headline workload:
    restarts from cells at depth >= branch_level run as a second pass in cell order.
    Times both forms on the same refreshed tree and checks that the targets agree."""
    dev = torch.device("cuda:0")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    msp.update_vacant_counts(tree, T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32))
    ty, va = T(w.neuron_type, torch.uint8), T(w.vac_axon, torch.int32)
    res = {}
    for b in (-1, branch_level):
        ms, info = [], {}
        for k in range(reps):
            tm = {}
            tgt, _ = msp.find_targets(tree, ty, va, w.sigma, w.theta, w.seed, w.step, timing=tm,
                                      branch_level=b, phase2=info)
            if k > 0:
                ms.append((tm["sweep_ms"], tm["draw_ms"] - tm["phase2_ms"], tm["phase2_ms"]))
        m = np.mean(np.array(ms), axis=0)
        res[b] = dict(sweep_ms=float(m[0]), draw_ms=float(m[1]), phase2_ms=float(m[2]),
                      requests=info["requests"], target=tgt.cpu().numpy())
    tree.free()
    one, two = res[-1], res[branch_level]
    kern_s = (two["sweep_ms"] + two["draw_ms"] + two["phase2_ms"]) / 1e3
    return dict(workload=w.name, searches=w.searches, branch_level=branch_level,
                second_phase_requests=two["requests"],
                request_bytes_paper_format=42 * two["requests"],
                one_phase_ms=dict(sweep=one["sweep_ms"], draw=one["draw_ms"]),
                two_phase_ms=dict(sweep=two["sweep_ms"], draw=two["draw_ms"],
                                  phase2=two["phase2_ms"]),
                identical_targets=bool(np.array_equal(one["target"], two["target"])),
                searches_per_s=w.searches / kern_s,
                roofline=alu_roofline(alg_ops, alg_bytes, kern_s, "level-0 vector operations "
                                      "of the one-phase search (the same lists) / the "
                                      "two-phase kernels' HIP-event time"),
                oracle="as cpu_baseline: the two-phase targets equal the one-phase ones",
                note="on one GPU the second phase only regroups work; the paper's gain is the "
                     "communication it removes between processes")


def bench_activity(msp, torch, w, steps=100):
    """Electrical activity between two connectivity updates (one epoch of `steps` 1 ms
    steps) on the synapses that one update of the headline workload forms, with every
    spike exchanged and with the firing-rate approximation between 8 ranks that own
    contiguous Morton ranges (the paper's domain division) or on every synapse."""
    dev = torch.device("cuda:0")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    ty = T(w.neuron_type, torch.uint8)
    va, ve, vi = (T(x, torch.int32) for x in (w.vac_axon, w.vac_exc, w.vac_inh))
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    msp.update_vacant_counts(tree, ve, vi)
    tgt, off = msp.find_targets(tree, ty, va, w.sigma, w.theta, w.seed, w.step)
    res = msp.commit_synapses(tgt, off, ty, va, ve, vi, w.seed, w.step, syn_capacity=w.searches)
    order = tree.export_topology()["order"]
    tree.free()
    rank = torch.empty(w.n, dtype=torch.int32, device=dev)
    rank[order.long()] = (torch.arange(w.n, device=dev) * 8 // w.n).to(torch.int32)
    src, tgt_, sty = res["syn_src"], res["syn_tgt"], res["syn_type"]
    m = src.numel()
    remote = float((rank[src.long()] != rank[tgt_.long()]).float().mean())
    out = dict(workload=f"activity_{w.n}_neurons_{m}_synapses", neurons=w.n, synapses=m,
               steps=steps, remote_synapse_share=remote)
    for approx, name in ((0, "exact"), (1, "approx_between_8_ranks"), (2, "approx_all")):
        a = msp.Activity(ty)
        a.run(src, tgt_, sty, seed=w.seed, t0=0, steps=steps, approx=approx, rank=rank)
        sp = torch.zeros(1, dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a.run(src, tgt_, sty, seed=w.seed, t0=steps, steps=steps, approx=approx, rank=rank,
              spikes=sp)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        # per step: the neuron state read and written (74 B per neuron); a spike sent
        # along an exact synapse (its index, target and type, the target's count: 13 B,
        # for the synapses of the neurons that fired); an approximated synapse (its
        # endpoints, type and the source's frequency: 17 B) and, with approx 1, the
        # rank-split flag of every synapse (1 B)
        n_apx = 0 if approx == 0 else (m * remote if approx == 1 else m)
        spikes_per_step = int(sp.item()) / steps
        sends = spikes_per_step * (m - n_apx) / w.n
        B = int(74 * w.n + 13 * sends + 17 * n_apx + (m if approx == 1 else 0))
        out[name] = dict(ms_per_step=sec * 1e3, neuron_steps_per_s=w.n / sec,
                         spikes=int(sp.item()), rate_hz=int(sp.item()) / w.n / (steps * 1e-3),
                         roofline=hbm_roofline(B, sec, "74 B per neuron + 13 B per spike sent "
                                               "along an exact synapse + 17 B per "
                                               "approximated synapse (+1 B per synapse, "
                                               "approx 1) and step / wall time per step"))
    # the oracle: 3 steps of the same network, all 8M neurons, one host thread
    from oracle import oracle as orc
    o = orc.Activity(w.neuron_type)
    hs, ht, hy = (x.cpu().numpy() for x in (src, tgt_, sty))
    t0 = time.perf_counter()
    o.run(hs, ht, hy, seed=w.seed, t0=0, steps=3)
    t_or = (time.perf_counter() - t0) / 3
    out["oracle"] = dict(value=w.n / t_or, unit="neuron steps/s", cores=1, kind="oracle",
                         sample="3 steps of the same network (every spike exchanged)")
    return out


def bench_batched(msp, torch, reps=5):
    """64 simulations of 2^12..2^18 neurons: one batched launch (HIP graph) against 64
    per-simulation find_targets calls, same stream, same results (checked)."""
    from synth_inputs import config_batched
    dev = torch.device("cuda:0")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    ws = config_batched()
    sims = []
    for k, w in enumerate(ws):
        tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
        msp.update_vacant_counts(tree, T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32))
        sims.append(dict(tree=tree, neuron_type=T(w.neuron_type, torch.uint8),
                         vac_axon=T(w.vac_axon, torch.int32), sigma=w.sigma, seed=w.seed + k))
    S = sum(w.searches for w in ws)
    log(f"batched: {len(ws)} simulations, {sum(w.n for w in ws)} neurons, {S} searches")
    b = msp.Batch(sims, graph=True, autotune=True)
    b.run(0.3, 0)                       # tunes, captures
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        b.run(0.3, r)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    assert b.status() == [0] * len(ws)
    bt = [b.results(k)[0].cpu().numpy().copy() for k in range(len(ws))]
    bufs = [torch.empty(max(w.searches, 1), dtype=torch.int32, device=dev) for w in ws]
    for d, buf in zip(sims, bufs):     # warm-up of the per-simulation path
        msp.find_targets(d["tree"], d["neuron_type"], d["vac_axon"], d["sigma"], 0.3, d["seed"],
                         reps - 1, target_out=buf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        outs = [msp.find_targets(d["tree"], d["neuron_type"], d["vac_axon"], d["sigma"], 0.3,
                                 d["seed"], r, target_out=buf)[0] for d, buf in zip(sims, bufs)]
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / reps
    same = all(np.array_equal(o.cpu().numpy(), x) for o, x in zip(outs, bt))
    b.free()
    B = ops = 0
    for k, d in enumerate(sims):
        cnt, off = counted(msp, d["tree"], d["neuron_type"], d["vac_axon"], d["sigma"], 0.3,
                           d["seed"], reps - 1)
        B += algorithmic_bytes(cnt, off)[0]
        ops += sweep_alu_ops(cnt, off)
    for d in sims:
        d["tree"].free()
    # the oracle on the simulations of up to 2^14 neurons, all of their searches
    from oracle import oracle as orc
    small = [(k, w) for k, w in enumerate(ws) if w.n <= (1 << 14)]
    t0 = time.perf_counter()
    S_small = 0
    for k, w in small:
        t = orc.OracleTree(w.pos, w.box_min, w.box_edge)
        t.update_counts(w.vac_exc, w.vac_inh)
        _, src, elem = orc.search_list(w.vac_axon)
        t.find_targets(w.neuron_type, w.sigma, 0.3, w.seed + k, 0, src, elem,
                       nthreads=oracle_threads())
        S_small += src.size
    t_or = time.perf_counter() - t0
    return dict(workload=f"batched_{len(ws)}_simulations", simulations=len(ws),
                neurons=int(sum(w.n for w in ws)), searches=int(S),
                batched_ms=tb * 1e3, batched_searches_per_s=S / tb,
                per_simulation_ms=tp * 1e3, per_simulation_searches_per_s=S / tp,
                speedup=tp / tb, identical_targets=bool(same),
                roofline=alu_roofline(ops, B, tb, "level-0 vector operations of all 64 "
                                      "searches / the batched launch's wall time"),
                oracle=dict(value=S_small / t_or, unit="searches/s",
                            cores=oracle_threads(), kind="oracle",
                            sample=f"all {S_small} searches of the {len(small)} simulations "
                                   f"with at most 16384 neurons, tree build and refresh "
                                   f"included"))


def bench_plasticity(msp, torch, updates=3):
    """The 100-update workload (2^23 neurons uniform in a 20,000 um cube), entirely on
    the device, run twice from the same start: (1) made of the separate calls, which
    read counts back between phases; (2) as update cycles (msp_cycle) replayed from a
    captured HIP graph, the host reading one status word per update. Each update
    refreshes the vacancies, searches and commits, then records the new synapses and
    runs the plasticity step (growth, deletion, retraction) that gives the next
    update's vacancies. The octree is built once (positions are fixed). Both runs must
    end in the same network."""
    from synth_inputs import config_large
    dev = torch.device("cuda:0")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    w = config_large()
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    ty = T(w.neuron_type, torch.uint8)
    ga, ge, gi = (T(v, torch.int32) for v in (w.vac_axon, w.vac_exc, w.vac_inh))
    net = msp.Network(ga, ge, gi, capacity=4 * w.n)
    per = []
    for step in range(updates):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        msp.update_vacant_counts(tree, ge, gi)
        tgt, off = msp.find_targets(tree, ty, ga, w.sigma, w.theta, w.seed, step)
        res = msp.commit_synapses(tgt, off, ty, ga, ge, gi, w.seed, step)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        net.record(res["syn_src"], res["syn_tgt"], res["syn_type"])
        ga, ge, gi = net.step(w.seed, step)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        S = int(off[-1].item())
        m = int(res["n_formed"])
        per.append(dict(update=step, searches=S, formed=m, synapses=net.m,
                        connectivity_ms=(t1 - t0) * 1e3, plasticity_ms=(t2 - t1) * 1e3,
                        searches_per_s=S / (t1 - t0)))
        if step < 3 or step % 10 == 9:
            log(f"plasticity update {step}: {S} searches, {m} formed, {net.m} synapses; "
                f"connectivity {(t1 - t0) * 1e3:.1f} ms, plasticity step "
                f"{(t2 - t1) * 1e3:.1f} ms")
    tot_s = sum(u["connectivity_ms"] + u["plasticity_ms"] for u in per) / 1e3
    searches = sum(u["searches"] for u in per)
    end_a = (net.m, int(net.bound.sum().item()), float(net.z.sum().item()))
    del net, res, tgt, off
    # the same updates as cycles replayed from one captured graph
    msp.release_workspace(0)
    va, ve, vi = (T(v, torch.int32) for v in (w.vac_axon, w.vac_exc, w.vac_inh))
    net = msp.Network(va, ve, vi, capacity=4 * w.n)
    cyc = msp.Cycle(tree, ty, net, va, ve, vi, w.sigma, w.theta, w.seed, step=0, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bad = 0
    for step in range(updates):
        cyc.run(1)
        bad |= cyc.status()              # the one host read of an update
    torch.cuda.synchronize()
    cyc_s = time.perf_counter() - t0
    c = cyc.counts()
    end_b = (c["m"], int(net.bound.sum().item()), float(net.z.sum().item()))
    log(f"plasticity: {updates} updates made of separate calls {tot_s:.3f} s, as replayed "
        f"update cycles {cyc_s:.3f} s; same network: {end_a == end_b}")
    cyc.free()
    tree.free()
    return dict(workload=f"plasticity_{w.n}_uniform_20000um", n_updates=len(per),
                total_s=tot_s, searches=searches, searches_per_s=searches / tot_s,
                cycle_graph_total_s=cyc_s, cycle_graph_searches_per_s=searches / cyc_s,
                cycle_status=bad, same_network=end_a == end_b,
                synapses_formed=sum(u["formed"] for u in per), synapses_at_end=end_a[0],
                first_updates=per[:3], last_update=per[-1],
                note="per update: refresh + search + commit, then record + growth/deletion/"
                     "retraction (the plasticity step), all on the device; octree built "
                     "once (positions fixed). total_s: the separate calls; "
                     "cycle_graph_total_s: the same updates replayed from a captured graph, "
                     "one status read per update")


def study_complexity(msp, torch, log2_ns=(12, 14, 16, 18, 20, 22, 23),
                     thetas=(0.2, 0.3, 0.4, 0.5)):
    """Visits per search and search throughput over n and theta at the density of the
    2^23-neuron workload (Sec. II: Barnes-Hut with theta > 0 needs O(log n) work per
    search). One JSON line per point, then a markdown table on stderr."""
    from synth_inputs import uniform_cube
    dev = torch.device("cuda:0")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    rows = []
    for lg in log2_ns:
        n = 1 << lg
        edge = 20000.0 * (n / float(1 << 23)) ** (1.0 / 3.0)
        w = uniform_cube(n, edge, seed=42)
        tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
        msp.update_vacant_counts(tree, T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32))
        ty, va = T(w.neuron_type, torch.uint8), T(w.vac_axon, torch.int32)
        S = w.searches
        buf = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
        for theta in thetas:
            _, off, _, _, cnt = msp.find_targets(tree, ty, va, w.sigma, theta, w.seed, 0,
                                                 target_out=buf, diag=True, counters=True)
            v = cnt["visits"].double().mean().item()
            v0 = cnt["visits0"].double().mean().item()
            ws = int(cnt["wave_steps"].item())
            v0h, offh = cnt["visits0"].cpu().numpy(), off.cpu().numpy()
            first = offh[:-1][np.diff(offh) > 0]          # one search per source
            lane_visits = int((v0h[first].astype(np.int64) - 1).sum())
            ms = []
            for _ in range(3):
                tm = {}
                msp.find_targets(tree, ty, va, w.sigma, theta, w.seed, 0, target_out=buf, timing=tm)
                ms.append(tm["kernel_ms"])
            t = float(np.median(ms))
            r = dict(study="complexity", n=n, edge_um=round(edge, 1), theta=theta, searches=S,
                     visits_per_search=v, level0_visits_per_search=v0,
                     lane_utilisation=lane_visits / max(1, 64 * ws), search_kernels_ms=t,
                     searches_per_s=S / (t * 1e-3))
            rows.append(r)
            print(json.dumps(r), flush=True)
        tree.free()
    log("| n | theta | visits/search | level-0 visits | lane utilisation | search ms | M searches/s |")
    log("|---:|---:|---:|---:|---:|---:|---:|")
    for r in rows:
        log(f"| {r['n']} | {r['theta']} | {r['visits_per_search']:.0f} | "
            f"{r['level0_visits_per_search']:.0f} | {r['lane_utilisation']:.2f} | "
            f"{r['search_kernels_ms']:.2f} | {r['searches_per_s'] / 1e6:.1f} |")


def bench_attraction(msp, torch, reps=5):
    """Expected attraction forward and adjoint (dL/dx, dL/dsigma of sum log Z) on 2^18
    neurons in a 5000 um cube."""
    from synth_inputs import config_attraction
    dev = torch.device("cuda:0")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    w = config_attraction()
    tree = msp.build_octree(T(w.pos, torch.float64), w.box_min, w.box_edge)
    msp.update_vacant_counts(tree, T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32))
    ty, va = T(w.neuron_type, torch.uint8), T(w.vac_axon, torch.int32)
    src = va > 0
    Z = msp.attraction_fwd(tree, ty, va, w.sigma, w.theta)
    gZ = torch.where(src, 1.0 / torch.where(src, Z, torch.ones_like(Z)), torch.zeros_like(Z))
    msp.attraction_bwd(tree, ty, va, w.sigma, w.theta, gZ)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        msp.attraction_fwd(tree, ty, va, w.sigma, w.theta)
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        msp.attraction_bwd(tree, ty, va, w.sigma, w.theta, gZ)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    cnt, off = counted(msp, tree, ty, va, w.sigma, w.theta, w.seed, 0)
    tree.free()
    ns = int(src.sum().item())
    Bf = sweep_bytes(cnt, off)
    first = off[:-1][np.diff(off) > 0]
    accepted = int(cnt["entries0"][first].astype(np.int64).sum())
    Bb = Bf + 24 * accepted              # plus one gradient (3 x float64) per accepted entry
    ops_f = sweep_alu_ops(cnt, off)
    # backward: the forward's operations plus, per accepted entry, the gradient
    # g w (2 / sigma^2) (x - c): 3 differences, 4 products
    ops_b = ops_f + 7 * accepted
    # the oracle (fp64, forward and analytic gradient) on a 32768-neuron cube at the
    # same density
    from oracle import oracle as orc
    from synth_inputs import uniform_cube
    wo = uniform_cube(32768, 5000.0 * (32768 / w.n) ** (1.0 / 3.0), seed=42)
    t0 = time.perf_counter()
    to = orc.OracleTree(wo.pos, wo.box_min, wo.box_edge)
    to.update_counts(wo.vac_exc, wo.vac_inh)
    to.attraction(wo.neuron_type, wo.vac_axon, wo.sigma, wo.theta, nthreads=oracle_threads())
    t_or = time.perf_counter() - t0
    return dict(workload=w.name, neurons=w.n, sources=ns, forward_ms=tf * 1e3,
                backward_ms=tb * 1e3, sources_per_s_forward=ns / tf,
                sources_per_s_backward=ns / tb,
                roofline_forward=alu_roofline(ops_f, Bf, tf, "level-0 vector operations / "
                                              "forward wall time"),
                roofline_backward=alu_roofline(ops_b, Bb, tb, "level-0 vector operations + 7 "
                                               "per accepted entry / backward wall time"),
                oracle=dict(value=int((wo.vac_axon > 0).sum()) / t_or, unit="sources/s",
                            cores=oracle_threads(), kind="oracle",
                            sample="forward and gradient of all sources of a 32768-neuron "
                                   "uniform cube at the same density (tree build included)"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["large", "clusters", "small"])
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--cpu-sample", type=int, default=400000)
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain-copy kernel used to scale HBM counters")
    ap.add_argument("--no-also", action="store_true",
                    help="skip the 2^20-neuron, batched, attraction and multi-update measurements")
    ap.add_argument("--study", choices=["complexity"], default=None,
                    help="instead of the benchmark: visits and throughput over n and theta")
    ap.add_argument("--updates", type=int, default=100,
                    help="updates of the multi-update workload measured with the others")
    ap.add_argument("--only", choices=["clusters", "batched", "attraction", "activity",
                                       "plasticity"], default=None,
                    help="instead of the benchmark: one of the other workloads alone (for "
                         "profiling), its result as one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding of the search is a design note, not implemented)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    if args.study == "complexity":
        import torch
        import paper_2509_26193_amd as msp
        study_complexity(msp, torch)
        return
    if args.only:
        import torch
        import paper_2509_26193_amd as msp
        if args.only == "clusters":
            from synth_inputs import config_clusters
            r = {f"theta{th}": bench_plain_update(msp, torch, config_clusters(theta=th),
                                                  steps=args.steps, warmup=args.warmup)
                 for th in (0.2, 0.3, 0.5)}
        elif args.only == "batched":
            r = bench_batched(msp, torch)
        elif args.only == "attraction":
            r = bench_attraction(msp, torch)
        elif args.only == "activity":
            r = bench_activity(msp, torch, make_workload("large", None))
        else:
            r = bench_plasticity(msp, torch, args.updates)
        print(json.dumps({"only": args.only, **r}), flush=True)
        return

    import torch
    import paper_2509_26193_amd as msp

    dev = torch.device("cuda:0")
    w = make_workload(args.workload, args.theta)
    S = w.searches
    log(f"workload {w.name}: n={w.n} searches={S} sigma={w.sigma} theta={w.theta}")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    pos = T(w.pos, torch.float64)
    ty = T(w.neuron_type, torch.uint8)
    va0, ve0, vi0 = T(w.vac_axon, torch.int32), T(w.vac_exc, torch.int32), T(w.vac_inh, torch.int32)
    va, ve, vi = va0.clone(), ve0.clone(), vi0.clone()
    tgt_buf = torch.empty(S, dtype=torch.int32, device=dev)
    off_buf = torch.empty(w.n + 1, dtype=torch.int64, device=dev)
    times = {"build": [], "refresh": [], "search": [], "commit": [], "sweep": [], "draw": []}

    def step(record):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        tree = msp.build_octree(pos, w.box_min, w.box_edge)
        ev[1].record()
        va.copy_(va0)
        ve.copy_(ve0)
        vi.copy_(vi0)
        msp.update_vacant_counts(tree, ve, vi)
        ev[2].record()
        tm = {}
        tgt, off = msp.find_targets(tree, ty, va, w.sigma, w.theta, w.seed, w.step,
                                    target_out=tgt_buf, elem_offset_out=off_buf, timing=tm)
        ev[3].record()
        res = msp.commit_synapses(tgt, off, ty, va, ve, vi, w.seed, w.step, syn_capacity=S)
        ev[4].record()
        tree.free()
        if record:
            # the phase events are read after the timed loop: no wait inside it
            pending.append(ev)
            times["sweep"].append(tm["sweep_ms"])
            times["draw"].append(tm["draw_ms"])
        return res["n_formed"]

    pending = []

    for k in range(args.warmup):
        step(False)
        log(f"warmup step {k + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    formed = 0
    for k in range(args.steps):
        formed = step(True)
        log(f"timed step {k + 1}/{args.steps}: sweep {times['sweep'][-1]:.2f} ms, "
            f"draw {times['draw'][-1]:.2f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps
    value = S / sec
    for ev in pending:
        for k, (a, b) in zip(("build", "refresh", "search", "commit"), zip(ev[:-1], ev[1:])):
            times[k].append(a.elapsed_time(b))

    # the last timed step's targets (the commit does not touch them): the cpu_baseline
    # leg compares them with the oracle
    gpu_target = tgt_buf[:S].cpu().numpy().astype(np.int64)

    # exact algorithmic work of the launch (the kernel's own counters, untimed pass)
    tree = msp.build_octree(pos, w.box_min, w.box_edge)
    va.copy_(va0); ve.copy_(ve0); vi.copy_(vi0)
    msp.update_vacant_counts(tree, ve, vi)
    tgt, off, cnt = msp.find_targets(tree, ty, va, w.sigma, w.theta, w.seed, w.step, counters=True)
    torch.cuda.synchronize()
    off_h = off.cpu().numpy()
    cnt_h = {k: v.cpu().numpy() for k, v in cnt.items()}
    counting_equal = bool(np.array_equal(tgt.cpu().numpy().astype(np.int64), gpu_target))
    tree.free()
    B, visits = algorithmic_bytes(cnt_h, off_h)
    first = off_h[:-1][np.diff(off_h) > 0]
    lane_steps = int((cnt_h["visits0"][first].astype(np.int64) - 1).sum())
    wave_steps = int(cnt_h["wave_steps"][0])
    union_eff = lane_steps / max(1, 64 * wave_steps)
    evals = int(cnt_h["entries0"][first].astype(np.int64).sum())
    ops = sweep_alu_ops(cnt_h, off_h)
    Bs = sweep_bytes(cnt_h, off_h)
    sweep_s = float(np.mean(times["sweep"])) / 1e3
    draw_s = float(np.mean(times["draw"])) / 1e3
    walk_bytes = WALK_REC_BYTES * wave_steps + WALK_SRC_BYTES * int(first.size)
    traffic = measured_traffic(w.name)
    issue = measured_counters(w.name)
    roof = dict(bound="alu", achieved=ops / sweep_s / 1e12, peak=VALU_OPS_PEAK / 1e12,
                unit="Tops/s", frac=ops / sweep_s / VALU_OPS_PEAK, traffic=traffic,
                kernel="search_sweep_k", kernel_ms=sweep_s * 1e3,
                ops_per_launch=ops,
                basis=(f"vector operations the method needs per source and level-0 record: "
                       f"{OPS_VISIT} per record with vacancy (squared distance, acceptance), "
                       f"{OPS_ENTRY} more per accepted entry (exp2, times v, running sum), "
                       f"{OPS_EMPTY} per record without; exact per-search counts of a counting "
                       f"launch; peak = 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz"),
                sweep_wave_steps=wave_steps, sweep_lane_visits=lane_steps,
                sweep_lane_utilisation=union_eff,
                timed_equals_counting_launch=counting_equal,
                # measured instruction issue of the sweep (committed rocprofv3 counters of
                # the same kernel sources, or null): vector-issue busy share and the share
                # of vector issue slots that do a lane's own work
                issue=None if issue is None else dict(
                    valu_insts=issue["SQ_INSTS_VALU"], salu_insts=issue["SQ_INSTS_SALU"],
                    kernel_ms=issue["kernel_ms"],
                    valu_busy=issue["SQ_INSTS_VALU"] * 4 / (1024 * 2.4e9 * issue["kernel_ms"] / 1e3),
                    useful_lane_issue=issue["SQ_INSTS_VALU"] * 4 / (1024 * 2.4e9 * issue["kernel_ms"] / 1e3)
                    * union_eff,
                    valu_per_wave_step=issue["SQ_INSTS_VALU"] / wave_steps,
                    salu_per_wave_step=issue["SQ_INSTS_SALU"] / wave_steps),
                # HBM views: the bytes the shared walk needs (one 32-byte record per wave
                # step, the sources' data and outputs), and the logical per-visit bytes
                # (16 B per lane visit, 8 B per open, 16 B per source: every lane charged
                # separately, so it exceeds 1 when the 64 lanes share a record load)
                hbm_shared_walk=dict(bytes=walk_bytes, achieved=walk_bytes / sweep_s / 1e9,
                                     unit="GB/s", frac=walk_bytes / sweep_s / HBM_PEAK),
                hbm_measured=None if traffic is None else dict(
                    bytes=traffic, achieved=traffic / sweep_s / 1e9, unit="GB/s",
                    frac=traffic / sweep_s / HBM_PEAK),
                logical_traversal=dict(bytes=Bs, achieved=Bs / sweep_s / 1e9, unit="GB/s",
                                       logical_traversal_frac=Bs / sweep_s / HBM_PEAK),
                search_total=dict(kernels="search_sweep_k+search_draw_k",
                                  ms=(sweep_s + draw_s) * 1e3, logical_bytes=B,
                                  node_visits=visits,
                                  logical_traversal_frac=B / (sweep_s + draw_s) / HBM_PEAK),
                # kernel evaluations at level 0 (entries of the accepted lists) per second
                # of the sweep, against the float32 exp2 rate (quarter rate)
                kernel_evals_per_s=evals / sweep_s, exp2_peak_per_s=EXP2_PEAK,
                exp2_frac=evals / sweep_s / EXP2_PEAK)
    log(f"step {sec * 1e3:.1f} ms; sweep {sweep_s * 1e3:.2f} ms ({roof['frac']:.3f} of the "
        f"vector-op peak, shared-walk HBM {roof['hbm_shared_walk']['frac']:.3f}); draw "
        f"{draw_s * 1e3:.2f} ms; {wave_steps} wave steps, lane utilisation {union_eff:.3f}; "
        f"timed targets equal the counting launch's: {counting_equal}")

    out = {
        "metric": "axon target searches/sec",
        "value": value,
        "unit": "searches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp64 (fp32 exp2 mantissa)",
        "data": "synthetic",
        "config": {"workload": w.name, "neurons": w.n, "searches_per_step": S,
                   "sigma_um": w.sigma, "theta": w.theta,
                   "step": "build_octree + update_vacant_counts + find_targets + commit_synapses",
                   "synapses_formed": formed},
        "breakdown_ms": {k: float(np.mean(v)) for k, v in times.items()},
        "search_kernels_searches_per_s": S / (sweep_s + draw_s),
        "roofline": roof,
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_also:
        from synth_inputs import config_clusters
        also = {}
        wc = config_clusters(theta=0.3)
        log(f"also: {wc.name}")
        also["plain_1M_clusters"] = bench_plain_update(msp, torch, wc, steps=5, warmup=1)
        del wc
        for th in (0.2, 0.5):             # the other thetas of the clustered workload
            wc = config_clusters(theta=th)
            log(f"also: {wc.name}")
            also[f"plain_1M_clusters_theta{th}"] = bench_plain_update(msp, torch, wc, steps=3,
                                                                      warmup=1)
            del wc
        log("also: two-phase search")
        also["two_phase_8M"] = bench_two_phase(msp, torch, w, B, ops)
        log("also: electrical activity")
        also["activity"] = bench_activity(msp, torch, w)
        log("also: batched")
        also["batched"] = bench_batched(msp, torch)
        log("also: attraction")
        also["attraction"] = bench_attraction(msp, torch)
        if args.updates > 0:
            log(f"also: {args.updates} updates of the multi-update workload")
            also["plasticity"] = bench_plasticity(msp, torch, args.updates)
        out["also"] = also
    if not args.no_cpu:
        threads = args.cpu_threads or oracle_threads()
        out["cpu_baseline"] = cpu_baseline(w, gpu_target, args.cpu_sample, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
