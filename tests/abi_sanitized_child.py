"""Child process of the sanitizer test (not collected by pytest): drives the C ABI of
an instrumented libmsp (path in argv[1]) through every argument check and handle
check that runs without a device, including handles that point at freed heap memory
and at foreign memory, and double frees. Exits 0 when every call returns the
documented status; a sanitizer report aborts the process."""
import ctypes
import sys

INVALID = -1

L = ctypes.CDLL(sys.argv[1])
libc = ctypes.CDLL(None)
libc.malloc.restype = ctypes.c_void_p
libc.malloc.argtypes = [ctypes.c_size_t]
libc.free.argtypes = [ctypes.c_void_p]

vp = ctypes.c_void_p
for name, res, args in [
    ("msp_status_string", ctypes.c_char_p, [ctypes.c_int32]),
    ("msp_octree_info", ctypes.c_int32, [vp, vp, vp]),
    ("msp_update_vacant_counts", ctypes.c_int32, [vp, vp, vp, vp]),
    ("msp_find_targets", ctypes.c_int32, [vp, vp, vp, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_uint64, ctypes.c_uint64, vp, vp,
                                          ctypes.c_int64, vp]),
    ("msp_last_device_error", ctypes.c_int32, [vp]),
    ("msp_octree_export_topology", ctypes.c_int32, [vp] * 8),
    ("msp_octree_export_aggregates", ctypes.c_int32, [vp, ctypes.c_int32, vp, vp, vp]),
    ("msp_attraction_fwd", ctypes.c_int32, [vp, vp, vp, ctypes.c_double, ctypes.c_double,
                                            vp, vp]),
    ("msp_free_octree", None, [vp]),
    ("msp_free_octree_async", ctypes.c_int32, [vp, vp]),
    ("msp_find_targets_batched", ctypes.c_int32, [vp, vp, ctypes.c_double, ctypes.c_uint64,
                                                  vp]),
    ("msp_batch_status", ctypes.c_int32, [vp, vp, vp]),
    ("msp_batch_free", None, [vp]),
    ("msp_batch_create", ctypes.c_int32, [vp, ctypes.c_int32, ctypes.c_int32, vp]),
    ("msp_build_octree", ctypes.c_int32, [vp, ctypes.c_int64, vp, ctypes.c_double,
                                          ctypes.c_int32, vp, vp]),
    ("msp_commit_synapses", ctypes.c_int32, [vp, vp, vp, ctypes.c_int64, vp, vp, vp,
                                             ctypes.c_uint64, ctypes.c_uint64, vp, vp, vp,
                                             ctypes.c_int64, vp, vp]),
    ("msp_search_offsets", ctypes.c_int32, [vp, ctypes.c_int64, vp, vp, vp]),
    ("msp_plasticity_step", ctypes.c_int32, [ctypes.c_int64, vp, ctypes.c_uint64,
                                             ctypes.c_uint64, vp, vp, vp, vp, vp,
                                             ctypes.c_int64, vp, vp, vp, vp, vp]),
    ("msp_plasticity_record", ctypes.c_int32, [ctypes.c_int64, vp, vp, vp, ctypes.c_int64,
                                               vp, vp, vp, ctypes.c_int64, ctypes.c_int64,
                                               vp, vp]),
    ("msp_activity_init", ctypes.c_int32, [ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
    ("msp_cycle_create", ctypes.c_int32, [vp, vp, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_uint64, vp, ctypes.c_int64, ctypes.c_int64,
                                          vp, ctypes.c_int32, vp]),
    ("msp_cycle_run", ctypes.c_int32, [vp, ctypes.c_int32, vp]),
    ("msp_cycle_free", None, [vp]),
]:
    f = getattr(L, name)
    f.restype = res
    f.argtypes = args

for st in range(-8, 2):
    assert L.msp_status_string(st)

# handles: never registered (a stack buffer), freed heap memory, null
foreign = ctypes.create_string_buffer(4096)
freed = libc.malloc(4096)
libc.free(freed)
handles = [ctypes.addressof(foreign), freed, None]
p8 = ctypes.c_void_p(8)
for h in handles:
    assert L.msp_octree_info(h, None, None) == INVALID
    assert L.msp_update_vacant_counts(h, p8, p8, None) == INVALID
    assert L.msp_find_targets(h, p8, p8, 750.0, 0.3, 1, 0, p8, p8, 10, None) == INVALID
    assert L.msp_last_device_error(h) == INVALID
    assert L.msp_octree_export_topology(h, *([None] * 7)) == INVALID
    assert L.msp_octree_export_aggregates(h, 0, None, None, None) == INVALID
    assert L.msp_attraction_fwd(h, p8, p8, 750.0, 0.3, p8, None) == INVALID
    assert L.msp_free_octree_async(h, None) == INVALID
    L.msp_free_octree(h)                   # a handle that is not live: nothing happens
    L.msp_free_octree(h)                   # ... also the second time
    assert L.msp_find_targets_batched(h, None, 0.3, 0, None) == INVALID
    assert L.msp_batch_status(h, None, None) == INVALID
    L.msp_batch_free(h)
    L.msp_batch_free(h)
    assert L.msp_cycle_run(h, 1, None) == INVALID
    L.msp_cycle_free(h)
    L.msp_cycle_free(h)

# argument checks before any device call
bm = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
out = ctypes.c_void_p()
assert L.msp_build_octree(None, 0, bm, 1.0, 1, None, ctypes.byref(out)) == INVALID
assert L.msp_build_octree(p8, 10, bm, 1.0, 2, None, ctypes.byref(out)) == INVALID
assert L.msp_build_octree(p8, 10, bm, float("inf"), 1, None, ctypes.byref(out)) == INVALID
assert L.msp_build_octree(p8, 1 << 40, bm, 1.0, 1, None, ctypes.byref(out)) == INVALID
assert L.msp_build_octree(p8, 10, None, 1.0, 1, None, ctypes.byref(out)) == INVALID
assert L.msp_build_octree(p8, 10, bm, 1.0, 1, None, None) == INVALID
assert L.msp_batch_create(None, 0, 0, ctypes.byref(out)) == INVALID
sims = ctypes.create_string_buffer(256)          # one msp_sim naming a foreign tree
ctypes.memmove(sims, ctypes.byref(ctypes.c_void_p(ctypes.addressof(foreign))), 8)
assert L.msp_batch_create(sims, 1, 0, ctypes.byref(out)) == INVALID
assert L.msp_commit_synapses(p8, None, p8, 10, p8, p8, p8, 1, 0, p8, p8, p8, 5, p8,
                             None) == INVALID
assert L.msp_commit_synapses(p8, p8, p8, 0, p8, p8, p8, 1, 0, p8, p8, p8, 5, p8,
                             None) == INVALID
assert L.msp_search_offsets(None, 10, p8, p8, None) == INVALID
assert L.msp_search_offsets(p8, 0, p8, p8, None) == INVALID
m_out = ctypes.c_int64(0)
assert L.msp_plasticity_step(0, p8, 1, 0, p8, p8, p8, p8, p8, 0, ctypes.byref(m_out), p8, p8,
                             p8, None) == INVALID
assert L.msp_plasticity_step(10, None, 1, 0, p8, p8, p8, p8, p8, 0, ctypes.byref(m_out), p8,
                             p8, p8, None) == INVALID
assert L.msp_plasticity_step(10, p8, 1, 0, p8, p8, p8, p8, p8, 1 << 31, ctypes.byref(m_out),
                             p8, p8, p8, None) == INVALID
assert L.msp_plasticity_record(0, p8, p8, p8, 1, p8, p8, p8, 0, 10, p8, None) == INVALID
assert L.msp_plasticity_record(10, p8, p8, p8, 20, p8, p8, p8, 0, 10, p8, None) == -4
assert L.msp_activity_init(0, p8, p8, p8, p8, p8, p8, p8, p8, None) == INVALID
assert L.msp_activity_init(10, p8, None, p8, p8, p8, p8, p8, p8, None) == INVALID
# the update cycle: a state with every pointer set, then each check in turn
state = (ctypes.c_void_p * 13)(*([8] * 13))
params = (ctypes.c_double * 6)(0.001, 0.7, 0.4, 0.7, 0.1, 0.1)
P = ctypes.create_string_buffer(bytes(params) + (100).to_bytes(4, "little") + bytes(4))
tree = ctypes.addressof(foreign)
assert L.msp_cycle_create(tree, p8, 750.0, 0.3, 1, P, 100, 100, state, 0,
                          ctypes.byref(out)) == INVALID          # not a live octree
assert L.msp_cycle_create(None, p8, 750.0, 0.3, 1, P, 100, 100, state, 0,
                          ctypes.byref(out)) == INVALID
assert L.msp_cycle_create(tree, p8, 750.0, 0.3, 1, P, 100, 100, None, 0,
                          ctypes.byref(out)) == INVALID
assert L.msp_cycle_create(tree, p8, 750.0, 0.3, 1, P, 100, 100, state, 0, None) == INVALID
assert out.value is None
print("abi checks under sanitizers: ok", flush=True)
