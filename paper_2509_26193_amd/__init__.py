"""MI355X (gfx950) implementation of the MSP connectivity update (arXiv 2509.26193).

The computation lives in libmsp.so (hand-written HIP kernels behind the C ABI of
include/msp.h); this package is its thin Python binding. Entry points follow the
four steps of one update: build_octree, update_vacant_counts, find_targets,
commit_synapses; Network holds the plasticity between updates and Cycle runs whole
updates without host waits.
"""
from ._lib import (ACTIVITY, PLASTICITY, Activity, AttractionFn, Batch, Cycle, MspError, Network, Octree,
                   attraction,
                   attraction_bwd, attraction_fwd, build_octree, commit_synapses, find_targets,
                   header_functions, lib, release_workspace, search_offsets, status_string, sync,
                   update_vacant_counts)

__all__ = ["AttractionFn", "attraction", "attraction_fwd", "attraction_bwd", "Batch", "MspError",
           "Octree", "build_octree", "update_vacant_counts", "find_targets",
           "commit_synapses", "Network", "Cycle", "PLASTICITY", "Activity", "ACTIVITY", "sync", "status_string",
           "header_functions", "lib", "search_offsets", "release_workspace"]
