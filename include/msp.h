/*
 * msp.h -- C ABI of libmsp, the MI355X (gfx950) implementation of the connectivity
 * update of the Model of Structural Plasticity with a Barnes-Hut target search,
 * as described in Czappa, Kaster, Wolf, "I Like To Move It -- Computation Instead
 * of Data in the Brain" (arXiv 2509.26193).
 *
 * The update (Sec. III-A, "Update of synapses"; Sec. III-B):
 *   1. msp_build_octree        -- spatial octree over the neurons (Sec. III-B,
 *                                 "Spatial octree"); positions never change, so once.
 *   2. msp_update_vacant_counts-- bottom-up vacancy aggregates (Sec. III-B,
 *                                 "Division of work"; Alg. 1, first three lines).
 *   3. msp_find_targets        -- every vacant axonal element draws a partner with
 *                                 the Barnes-Hut acceptance test and restarts
 *                                 (Sec. III-B, "Division of work").
 *   4. msp_commit_synapses     -- each neuron accepts as many requests as it has
 *                                 vacant dendritic elements, at random; the rest are
 *                                 declined (Sec. III-A, "Update of synapses").
 * Around it: the batched search of many simulations (msp_batch_*), the expected
 * attraction and its adjoint (msp_attraction_*), the change of the network between
 * updates (msp_plasticity_*), the two-phase search of Sec. IV-A (branch_level of
 * msp_find_targets_diag) and the electrical activity with the firing-rate
 * approximation of Sec. IV-B (msp_activity_run).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller unless marked (host).
 *     The caller keeps them alive until the work queued on the stream has finished.
 *   - Work is queued on the given stream `s` (0 = the default stream). Calls that
 *     must size something or report an error found on the device (build,
 *     find_targets, commit, the plasticity step, the activity run) read values back
 *     to the host and therefore wait on `s`, as each one states; the others are
 *     asynchronous.
 *   - Every call returns an msp_status and never throws. Arguments are validated
 *     before anything is queued; on an error nothing is written.
 *   - Data-dependent errors found on the device (a non-finite position, a negative
 *     count) raise a sticky per-octree flag read by msp_last_device_error.
 *   - Neuron ids are 0..n-1, the row order of the position array. Neuron type 0 =
 *     excitatory, 1 = inhibitory. A source of type t searches the type-t vacant
 *     dendritic elements (the request carries the cell type, Sec. III-B).
 *   - Limits: 1 <= n <= MSP_MAX_NEURONS; the octree has fewer than 2^26 nodes.
 */
#ifndef MSP_H
#define MSP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t msp_status;
#define MSP_OK                 0
#define MSP_ERR_INVALID       (-1)  /* bad argument; a handle that is not live        */
#define MSP_ERR_OOM           (-2)  /* device allocation failed                       */
#define MSP_ERR_HIP           (-3)  /* a HIP runtime call failed                      */
#define MSP_ERR_CAPACITY      (-4)  /* an output buffer is too small; nothing written */
#define MSP_ERR_DEVICE        (-5)  /* data error detected on the device              */
#define MSP_ERR_UNIMPLEMENTED (-6)
#define MSP_ERR_TOO_LARGE     (-7)  /* beyond the fixed working memory of an
                                       allocation-free entry point                   */

#define MSP_MAX_NEURONS (1LL << 25)

typedef struct msp_octree_s* msp_octree;

/*
 * Build the octree over n neurons (Sec. III-B, "Spatial octree"; "Division of the
 * simulation domain" for the Morton-indexed cells).
 *   pos       [n][3] float64, row-major (x, y, z) per neuron, micrometres.
 *   box_min   (host) [3] minimum corner of the cubic domain; box_edge (host) its edge,
 *             in [2^-480, 2^480]. Each axis is quantised to 21 bits,
 *             q = floor((x - min) / edge * 2^21), clamped into [0, 2^21 - 1] (positions
 *             outside the cube fall in edge cells).
 *   leaf_size must be 1: a leaf holds one neuron, except that neurons whose quantised
 *             positions coincide share one depth-21 leaf.
 *   out       (host) receives the handle. The library owns every node array.
 * Errors: MSP_ERR_INVALID for n < 1 or n > MSP_MAX_NEURONS, a non-finite box corner, an
 * edge outside that range, leaf_size != 1, null pointers; MSP_ERR_OOM. A non-finite
 * position sets the device error flag. The build waits on `s` twice (to size the node
 * arrays and the per-depth lists); its last kernels may still run when it returns.
 */
msp_status msp_build_octree(const double* pos, int64_t n, const double box_min[3],
                            double box_edge, int32_t leaf_size, hipStream_t s,
                            msp_octree* out);

/*
 * Refresh the per-type vacancy aggregates bottom-up (Sec. III-B, "Division of work":
 * a leaf carries its neuron's position and count, an inner node the sum of its
 * children's counts and the count-weighted average of their positions).
 *   vac_dend_exc, vac_dend_inh [n] int32 >= 0, vacant dendritic elements per neuron.
 * Centroids are accumulated in float64 over the children in octant order, one
 * rounding per operation. Idempotent; topology is unchanged. A negative count sets
 * the device error flag.
 */
msp_status msp_update_vacant_counts(msp_octree t, const int32_t* vac_dend_exc,
                                    const int32_t* vac_dend_inh, hipStream_t s);

/*
 * Barnes-Hut target search for every vacant axonal element (Sec. III-B, "Division
 * of work"; Sec. III-A, "Update of synapses").
 *   neuron_type [n] uint8 (0/1); vac_axon [n] int32, a_i >= 0 searches of neuron i.
 *   sigma_um > 0: kernel width, weight of a node = v * exp(-d^2 / sigma^2).
 *   theta >= 0: a cell of edge l at distance d from the source is accepted iff
 *             l < theta * d (evaluated as l*l < theta*theta*d*d in float64); leaves are
 *             always accepted, a cell containing the source is always opened.
 *   seed, step: the draw of element j of neuron i at restart level k uses Philox4x64-10
 *             with key (seed, 0) and counter (i, j, step, k).
 *   target_out [capacity_S] int32: target_out[elem_offset[i] + j] = chosen neuron id,
 *             or -1 if no neuron with a vacancy of the right type has nonzero weight.
 *   elem_offset_out [n+1] int64: exclusive prefix sum of vac_axon (CSR by source).
 * Every search reads the octree as refreshed last (all requests are formed before
 * any is answered). The level-0 normaliser Z of a source (Sec. III-A) is added up in
 * float64 in the walk's depth-first order; a call with few sources (under 2^21) cuts
 * the walk into up to 8 consecutive pre-order ranges, searched in parallel, whose sums
 * are then added in order, so Z's last bits depend on the cut (the draw follows the
 * same sums). Errors: MSP_ERR_CAPACITY if S = sum(vac_axon) > capacity_S:
 * then only elem_offset_out is written (elem_offset_out[n] = S sizes the buffer);
 * MSP_ERR_INVALID for sigma <= 0, theta < 0, a negative vac_axon or a type > 1
 * (the last two found on the device before the search: target_out is not written).
 * Working memory: about 200 B per neuron plus the search checkpoints, up to 3 KB per
 * neuron but never more than an eighth of the device's memory. The library keeps it
 * per device between calls and grows it when a larger search needs more (it is held
 * until msp_release_workspace or the end of the process; MSP_ERR_OOM if it cannot be
 * had). Searches on one device take turns with it: a call holds it from entry to
 * return, and the kernels of a call on another stream wait for those of the previous
 * call. The call waits on `s` once, after the worklist is built, to read the status.
 */
msp_status msp_find_targets(msp_octree t, const uint8_t* neuron_type, const int32_t* vac_axon,
                            double sigma_um, double theta, uint64_t seed, uint64_t step,
                            int32_t* target_out, int64_t* elem_offset_out, int64_t capacity_S,
                            hipStream_t s);

/*
 * msp_find_targets without any memory allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid device
 * allocation). Same arguments, results and errors as msp_find_targets (targets
 * bitwise equal), one phase, no diagnostics. Its working memory is one fixed array
 * per device inside the library's code object (40 MiB, held by every device the
 * library runs on until the process ends), enough for n <= MSP_NOALLOC_MAX_NEURONS;
 * a larger octree returns MSP_ERR_TOO_LARGE before anything is queued, and a call
 * while another device than the octree's is current MSP_ERR_INVALID. Every call on
 * one device shares that array: calls that overlap on a device (on different
 * streams, or from different host threads) race and must be ordered by the caller.
 * The call waits on `s` once, after the worklist is built, to read the status.
 */
#define MSP_NOALLOC_MAX_NEURONS (1LL << 16)
msp_status msp_find_targets_noalloc(msp_octree t, const uint8_t* neuron_type,
                                    const int32_t* vac_axon, double sigma_um, double theta,
                                    uint64_t seed, uint64_t step, int32_t* target_out,
                                    int64_t* elem_offset_out, int64_t capacity_S, hipStream_t s);

/*
 * The searches msp_find_targets will run, so that a caller can size target_out:
 * elem_offset_out [n+1] int64 = exclusive prefix sum of vac_axon [n] int32 (CSR by
 * source, as msp_find_targets writes it) and *S_out (host) = elem_offset_out[n].
 * MSP_ERR_INVALID for n < 1 or n > MSP_MAX_NEURONS, a null pointer, or a negative
 * count (found on the device; it counts as 0 in the offsets). Waits on `s`.
 */
msp_status msp_search_offsets(const int32_t* vac_axon, int64_t n, int64_t* elem_offset_out,
                              int64_t* S_out, hipStream_t s);

/*
 * Diagnostics of one msp_find_targets call. Every pointer is nullable.
 *   z0      [S] float64: normaliser of the level-0 list of each search;
 *   levels  [S] int32: number of lists drawn from (1 + restarts);
 *   visits  [S] int32: node records examined over all levels (a start node counts
 *           once, a bucket leaf once); opens [S] int32: nodes replaced by their
 *           children over all levels (the start node included);
 *   visits0, opens0 [S] int32: the level-0 part of visits / opens (the level-0 list
 *           of a source is shared by all of its elements);
 *   kernel_ms (host) [3]: durations in ms, from HIP events recorded on `s` around each
 *           kernel: [0] the level-0 sweep, [1] the draws and restarts of the first
 *           phase, [2] the second phase (0 with one phase); when set, the call waits
 *           for the kernels to finish.
 *   wave_steps (device int64 scalar): incremented by the number of node steps of the
 *           shared level-0 walks (one per 64-source wavefront tile); with visits0 it
 *           gives the fraction of lanes doing useful work. Counted only when one of
 *           the per-search arrays above is also requested.
 *   branch_level: the two-phase (location-aware) form of the search (Sec. IV-A).
 *           Restarts from a drawn cell at depth >= branch_level (1..21) are not run
 *           where they are drawn: they become requests (source, element, cell, level)
 *           that a second pass runs in cell order, which groups them by branch cell
 *           (depth-b subtree) as the paper groups them by owning process. Targets,
 *           levels, visits and opens are bitwise those of the one-phase search.
 *           0: the library's default (one phase); above 21 or negative: one phase.
 *           The second phase needs about 40 B per search of working memory.
 *   phase2_requests (device int64 scalar): set to the number of second-phase requests.
 *   parts_per_tile: 0 (the default): the library's choice; 1, 2, 4 or 8: every tile's
 *           level-0 walk is cut into this many parts (see msp_find_targets); other
 *           values are MSP_ERR_INVALID. Visits and opens do not depend on it; z0 does
 *           in its last bits only.
 *   entries0 [S] int32: the number of entries of the level-0 accepted list (cells
 *           accepted and neurons listed: the kernel evaluations of the level-0 sum).
 */
typedef struct msp_search_diag {
  double* z0;
  int32_t* levels;
  int32_t* visits;
  int32_t* opens;
  int32_t* visits0;
  int32_t* opens0;
  float* kernel_ms;
  int64_t* wave_steps;
  int32_t branch_level;
  int64_t* phase2_requests;
  int32_t parts_per_tile;
  int32_t* entries0;
} msp_search_diag;

/* msp_find_targets with diagnostics (diag may be null). */
msp_status msp_find_targets_diag(msp_octree t, const uint8_t* neuron_type,
                                 const int32_t* vac_axon, double sigma_um, double theta,
                                 uint64_t seed, uint64_t step, int32_t* target_out,
                                 int64_t* elem_offset_out, int64_t capacity_S,
                                 const msp_search_diag* diag, hipStream_t s);

/*
 * Batched search: many independent simulations (each with its own octree, built and
 * refreshed as above, and its own sources, kernel width, seed and outputs) searched
 * by one set of launches. Per simulation the result is bitwise equal to
 * msp_find_targets with the same arguments. Intended for ensembles of simulations
 * too small to fill the GPU one at a time.
 *
 * A plan fixes the simulations' octrees (their sizes determine its scratch, which
 * the plan owns: a run allocates nothing and does not synchronise with the host).
 * Each run may pass new buffers, kernel widths and seeds for the same octrees.
 */
typedef struct msp_sim {
  msp_octree tree;
  const uint8_t* neuron_type;   /* [n] device */
  const int32_t* vac_axon;      /* [n] device */
  double sigma_um;              /* > 0 */
  uint64_t seed;                /* Philox key word 0 of this simulation's draws */
  int32_t* target_out;          /* [capacity_S] device */
  int64_t* elem_offset_out;     /* [n + 1] device */
  int64_t capacity_S;
} msp_sim;

typedef struct msp_batch_s* msp_batch;

#define MSP_BATCH_GRAPH    1    /* capture the launches in a HIP graph on the first run,
                                   replay it afterwards */
#define MSP_BATCH_AUTOTUNE 2    /* on the first run, time several launch shapes (sweep
                                   occupancy, draw block size, checkpoint slots per
                                   region; each the median of 3 timed runs) and keep
                                   the fastest (the targets do not depend on them) */

/* Create a plan over n_sims >= 1 simulations on the current device (host array sims,
 * copied). Errors: MSP_ERR_INVALID (bad handle, unrefreshed octree, bad sigma,
 * n_sims < 1), MSP_ERR_OOM. */
msp_status msp_batch_create(const msp_sim* sims, int32_t n_sims, int32_t flags, msp_batch* out);

/* Run the batched search on stream s with a shared theta and step. `sims` (host,
 * nullable = reuse the previous run's) must name the plan's octrees in the same order.
 * Asynchronous: per-simulation errors (capacity exceeded, negative vac_axon, type > 1)
 * are reported by msp_batch_status; such a simulation's target_out is not written, its
 * elem_offset_out is. A run without `sims` writes the new theta and step on the device
 * and never waits; a run with `sims` (and the first run) uploads the descriptors from
 * a host staging buffer and first waits until the previous upload has been read.
 * Runs of one plan must be ordered (one stream, or ordered by the caller). */
msp_status msp_find_targets_batched(msp_batch b, const msp_sim* sims, double theta,
                                    uint64_t step, hipStream_t s);

/* Wait for the last run on stream s and copy the per-simulation status to status_out
 * (host [n_sims]; MSP_OK, MSP_ERR_CAPACITY or MSP_ERR_INVALID each). Returns MSP_OK if
 * every simulation succeeded, else the first failing status. */
msp_status msp_batch_status(msp_batch b, hipStream_t s, int32_t* status_out);

/* Release the plan (waits for the device). */
void msp_batch_free(msp_batch b);

/*
 * Expected attraction (the differentiated form). For every neuron i with vac_axon > 0,
 * Z_out[i] = the normaliser of its level-0 Barnes-Hut list: the sum over the accepted
 * cells and neurons e (type of i, acceptance as in msp_find_targets) of
 * v_e * exp(-|x_i - c_e|^2 / sigma^2); Z_out[i] = 0 for the other neurons. float32
 * output, float64 accumulation. The octree must be refreshed; its positions are the
 * positions differentiated.
 */
msp_status msp_attraction_fwd(msp_octree t, const uint8_t* neuron_type, const int32_t* vac_axon,
                              double sigma_um, double theta, float* Z_out, hipStream_t s);

/*
 * Adjoint of msp_attraction_fwd with every acceptance decision held fixed (the
 * function is piecewise smooth in the positions): given gZ[n] = dLoss/dZ_i (float32,
 * entries of neurons without vacant axonal elements are ignored), writes
 * dpos[n][3] = dLoss/dx (float32) and dsigma (device float64 scalar) = dLoss/dsigma.
 * Centroid gradients reach the neurons of a cell as v_j / v_C. Uses float64 atomics:
 * the result is deterministic up to the order of floating-point additions.
 */
msp_status msp_attraction_bwd(msp_octree t, const uint8_t* neuron_type, const int32_t* vac_axon,
                              double sigma_um, double theta, const float* gZ, float* dpos,
                              double* dsigma, hipStream_t s);

/*
 * Accept or decline every request (Sec. III-A, "Update of synapses"; Sec. III-B:
 * requests are exchanged, accepted locally and answered yes/no).
 *   target [S], elem_offset [n+1]: as produced by msp_find_targets.
 *   Requests on target g of source type t form one group; the group accepts
 *   min(#requests, vacant type-t dendritic elements of g) requests, those with the
 *   smallest Philox4x64-10 word 0 under key (seed, 1) and counter (i, j, step, 0),
 *   ties broken by (i, j); the rest are declined.
 *   vac_axon, vac_exc, vac_inh [n] int32, in/out: decremented by the synapses formed.
 *   syn_src, syn_tgt [syn_capacity] int32, syn_type [syn_capacity] uint8: the formed
 *   synapses, ordered by (source, element). n_formed: device int64 scalar.
 *   accepted_out [S] uint8 (nullable in msp_commit_synapses_ex): 1 if the request in
 *   that slot was accepted.
 * Errors: MSP_ERR_CAPACITY if more than syn_capacity synapses would form, and
 * MSP_ERR_INVALID if a target is >= n (then no vacancy count is modified, no synapse is
 * written and *n_formed = 0); MSP_ERR_INVALID if S = elem_offset[n] is negative or
 * not below 2^31 - 1 (requests are indexed with int32). Waits on `s` (to size its
 * working memory by S and to report the status). The working memory (about 40 B per
 * request and 24 B per neuron) is the one the library keeps per device for searches
 * (see msp_find_targets): commits and searches on one device take turns with it.
 * After a commit the octree is stale until the next msp_update_vacant_counts.
 */
msp_status msp_commit_synapses(const int32_t* target, const int64_t* elem_offset,
                               const uint8_t* neuron_type, int64_t n, int32_t* vac_axon,
                               int32_t* vac_exc, int32_t* vac_inh, uint64_t seed, uint64_t step,
                               int32_t* syn_src, int32_t* syn_tgt, uint8_t* syn_type,
                               int64_t syn_capacity, int64_t* n_formed, hipStream_t s);

msp_status msp_commit_synapses_ex(const int32_t* target, const int64_t* elem_offset,
                                  const uint8_t* neuron_type, int64_t n, int32_t* vac_axon,
                                  int32_t* vac_exc, int32_t* vac_inh, uint64_t seed,
                                  uint64_t step, int32_t* syn_src, int32_t* syn_tgt,
                                  uint8_t* syn_type, int64_t syn_capacity, int64_t* n_formed,
                                  uint8_t* accepted_out, hipStream_t s);

/* Release the octree (waits for the device to finish using it). The library keeps a
 * registry of the handles it has handed out and never reads through a handle that is
 * not in it: every call rejects a freed or foreign handle with MSP_ERR_INVALID, and a
 * second free of the same handle does nothing. */
void msp_free_octree(msp_octree t);

/* Stream-ordered release: the octree's memory returns to the library's pool after the
 * work queued on `s` so far; the handle is invalid at once. The caller orders every
 * other use of the octree (on other streams) before that point. MSP_ERR_INVALID for
 * a handle that is not live. */
msp_status msp_free_octree_async(msp_octree t, hipStream_t s);

/* Free the working memory the library keeps on `device` for searches, commits and
 * plasticity steps (see msp_find_targets), after the last call that used it has
 * finished (waits for it). The next such call on that device allocates it again. MSP_ERR_INVALID for a device that does not
 * exist. */
msp_status msp_release_workspace(int32_t device);

/* Wait for stream s; MSP_ERR_HIP if the stream reported an error. */
msp_status msp_sync(hipStream_t s);

/* Static description of a status code. */
const char* msp_status_string(msp_status st);

/* Synchronise on the device and return MSP_ERR_DEVICE if a data error (non-finite
 * position at build, negative count at refresh) was detected, else MSP_OK. Clears
 * nothing: the flag is sticky for the life of the octree. */
msp_status msp_last_device_error(msp_octree t);

/* Sizes: number of neurons and nodes (host outputs, nullable). */
msp_status msp_octree_info(msp_octree t, int64_t* n_neurons, int64_t* n_nodes);

/*
 * Copy the topology out (all outputs device pointers, nullable):
 *   order [n] int32 neuron ids in (Morton key, id) order; keys [n] uint64 sorted keys;
 *   depth [N] int32; node_begin, node_end [N] int64 ranges into `order`;
 *   subtree_end [N] int64: nodes are numbered in depth-first pre-order, children in
 *   octant order (digit 4x + 2y + z), so the subtree of node k is [k, subtree_end[k]).
 */
msp_status msp_octree_export_topology(msp_octree t, int32_t* order, uint64_t* keys,
                                      int32_t* depth, int64_t* node_begin, int64_t* node_end,
                                      int64_t* subtree_end, hipStream_t s);

/* Copy the type-`type` aggregates out: count [N] int64, centroid [N][3] float64 (device,
 * nullable). The centroid of a node with count 0 is unspecified. */
msp_status msp_octree_export_aggregates(msp_octree t, int32_t type, int64_t* count,
                                        double* centroid, hipStream_t s);

/* ------------------------------------------------------------------------------------
 * Plasticity between connectivity updates (Sec. III-A, "Update of synaptic elements"
 * and the first sub-phase of "Update of synapses"): the element counts of every
 * neuron grow or retract with its calcium, synapses are deleted at random, and
 * retracted elements that were bound break random synapses. With these two calls the
 * whole multi-update loop stays on the device.
 *
 * State (device, owned by the caller):
 *   z [3][n] float64: continuous element counts, kinds 0 axon, 1 excitatory dendrite,
 *     2 inhibitory dendrite;
 *   bound [3][n] int32: elements of each kind bound in synapses;
 *   syn_src, syn_tgt [m] int32 and syn_type [m] uint8 (0 excitatory, 1 inhibitory: the
 *     source's type): the synapse list, in the order the synapses were recorded. A
 *     synapse (i, g, type) binds one axonal element of i and one dendritic element of
 *     kind 1 + type of g.
 * ------------------------------------------------------------------------------------ */
typedef struct msp_plasticity_params {
  double growth_rate;       /* nu: element growth per simulation step at the peak */
  double target_calcium;    /* eps: calcium at which elements neither grow nor retract */
  double growth_onset;      /* eta: calcium below which elements retract */
  double calcium_mean;      /* calcium is drawn from N(calcium_mean, calcium_sd) */
  double calcium_sd;
  double delete_fraction;   /* share of the synapses deleted at random per update */
  int32_t steps_per_update; /* simulation steps between two connectivity updates */
} msp_plasticity_params;

/*
 * Append m_new synapses (device arrays new_src, new_tgt, new_type, e.g. a commit's
 * output) at [m, m + m_new) of the list and bind their elements in bound [3][n].
 * Errors: MSP_ERR_CAPACITY if m + m_new > capacity (nothing written); MSP_ERR_INVALID
 * for n < 1, m < 0, m_new < 0, or a neuron id outside [0, n) or a type > 1 (found on
 * the device: the list is appended but such a synapse binds nothing). Waits on `s`.
 */
msp_status msp_plasticity_record(int64_t n, const int32_t* new_src, const int32_t* new_tgt,
                                 const uint8_t* new_type, int64_t m_new, int32_t* syn_src,
                                 int32_t* syn_tgt, uint8_t* syn_type, int64_t m, int64_t capacity,
                                 int32_t* bound, hipStream_t s);

/*
 * One step between update `step` and the next, in this order:
 *   1. growth: calcium Ca of neuron j, kind k = calcium_mean + calcium_sd * G, G from
 *      Box-Muller on words 0 and 1 of Philox4x64-10 with key (seed, 2) and counter
 *      (j, k, step, 0): u1 = ((w0 >> 11) + 1) 2^-53, u2 = (w1 >> 11) 2^-53,
 *      G = sqrt(-2 ln u1) cos(2 pi u2); then z += steps * nu * (2 exp(-((Ca - xi) /
 *      zeta)^2) - 1), xi = (eta + eps) / 2, zeta = (eps - eta) / (2 sqrt(ln 2)), and z
 *      is clamped at 0;
 *   2. deletion: the floor(delete_fraction * m + 0.5) synapses of smallest (word 0 of
 *      Philox key (seed, 3), counter (s, step, 0, 0); then s) are deleted, s being the
 *      synapse's place in the list at the start of the step;
 *   3. retraction, for kinds k = 0, 1, 2 in turn: a neuron with bound > floor(z) of
 *      kind k loses that many of its synapses of that kind, those of smallest (top 32
 *      bits of word 0 of Philox key (seed, 4), counter (s, step, k, 0); then s);
 *   4. the list is compacted in order; *m_out (host) = its new length;
 *   5. vac_axon, vac_exc, vac_inh [n] int32 = floor(z) - bound of each kind.
 * Errors: MSP_ERR_INVALID for n < 1, m < 0 or m >= 2^31, a null pointer or parameters
 * that are not finite (or growth_onset >= target_calcium). Waits on `s`. Its working
 * memory (about 60 B per synapse) is the one the library keeps per device for
 * searches (see msp_find_targets).
 */
msp_status msp_plasticity_step(int64_t n, const msp_plasticity_params* params, uint64_t seed,
                               uint64_t step, double* z, int32_t* bound, int32_t* syn_src,
                               int32_t* syn_tgt, uint8_t* syn_type, int64_t m, int64_t* m_out,
                               int32_t* vac_axon, int32_t* vac_exc, int32_t* vac_inh,
                               hipStream_t s);

/* ------------------------------------------------------------------------------------
 * The update cycle (Sec. III-A: every connectivity update refreshes the octree's
 * vacancy counts, searches a target for every vacant axonal element, accepts or
 * declines the requests, records the new synapses, and the elements then grow,
 * retract and are deleted until the next update). msp_cycle_run enqueues whole
 * updates with every count kept on the device: nothing is read back and nothing is
 * allocated, so the host never waits inside an update and, with MSP_CYCLE_GRAPH, one
 * update is captured as a HIP graph and replayed. An update does exactly what
 *   msp_update_vacant_counts(t, vac_exc, vac_inh),
 *   msp_find_targets(t, neuron_type, vac_axon, sigma, theta, seed, step, ...),
 *   msp_commit_synapses(..., seed, step, ...), msp_plasticity_record(...),
 *   msp_plasticity_step(n, params, seed, step, ...)
 * do in turn with step = *state.step, then increments *state.step: the network state
 * it leaves is bitwise the same.
 * ------------------------------------------------------------------------------------ */
typedef struct msp_cycle_s* msp_cycle;

/* The network state an update cycle reads and advances: device memory owned by the
 * caller, which must stay valid until msp_cycle_free. */
typedef struct msp_cycle_state {
  double* z;             /* [3][n] element counts (kinds as in msp_plasticity_step) */
  int32_t* bound;        /* [3][n] bound elements */
  int32_t* syn_src;      /* [syn_capacity] the synapse list */
  int32_t* syn_tgt;
  uint8_t* syn_type;
  int64_t* m;            /* [1] synapses in the list */
  int32_t* vac_axon;     /* [n] vacant elements: the update's input, rewritten by its */
  int32_t* vac_exc;      /*     plasticity step for the next update */
  int32_t* vac_inh;
  uint64_t* step;        /* [1] step of the next update; incremented by every update */
  int32_t* status;       /* [1] MSP_CYCLE_* bits, OR-ed in by every update (the caller
                            clears it) */
  int64_t* searches;     /* [1] nullable: searches of the last update */
  int64_t* formed;       /* [1] nullable: synapses formed by the last update */
} msp_cycle_state;

#define MSP_CYCLE_GRAPH 1       /* capture one update on the first run, replay it after */

/* status bits of an update (device) */
#define MSP_CYCLE_SEARCH_INVALID  1   /* a negative vac_axon or a neuron type > 1: the
                                         update searched nothing and formed nothing */
#define MSP_CYCLE_SEARCH_CAPACITY 2   /* more searches than search_capacity: likewise */
#define MSP_CYCLE_SYN_CAPACITY    4   /* the list could not hold the new synapses: none
                                         was recorded (their elements stay unbound) */
#define MSP_CYCLE_DEVICE          8   /* the octree's device error flag is set (e.g. a
                                         negative vacant dendritic count) */

/* Plan update cycles of the network on octree t (built; its positions are the
 * neurons'), neuron_type [n], on the current device (t's). search_capacity: most
 * searches one update may run (the sum of vac_axon); syn_capacity: the list's length.
 * The plan holds its own working memory (search, acceptance and plasticity scratch,
 * sized by n, search_capacity and syn_capacity). Errors: MSP_ERR_INVALID (bad handle,
 * null state pointer, sigma or theta, parameters as msp_plasticity_step checks them,
 * search_capacity < 1 or not below 2^31 - 1, syn_capacity < 1 or not below 2^31),
 * MSP_ERR_OOM. */
msp_status msp_cycle_create(msp_octree t, const uint8_t* neuron_type, double sigma_um,
                            double theta, uint64_t seed, const msp_plasticity_params* params,
                            int64_t search_capacity, int64_t syn_capacity,
                            const msp_cycle_state* state, int32_t flags, msp_cycle* out);

/* Enqueue `updates` >= 0 consecutive updates on stream s. Does not wait: read
 * *state.status (and the state) after the stream has reached them. */
msp_status msp_cycle_run(msp_cycle c, int32_t updates, hipStream_t s);

/* Release the plan (waits for the device). */
void msp_cycle_free(msp_cycle c);

/*
 * Electrical activity between connectivity updates (Sec. II, "Update of electrical
 * activity") with the firing-rate approximation of Sec. IV-B: neurons exchange
 * spikes, integrate them and their background input, record new spikes and update
 * their calcium; every epoch of `epoch` steps their firing frequency is refreshed.
 * Parameters of the neuron model (Izhikevich 2003: a, b, c, d per type, regular
 * spiking for excitatory and fast spiking for inhibitory neurons), the synaptic
 * weights per received spike, the uniform background current (mean, width) and the
 * calcium increment per spike and time constant (in steps):
 */
typedef struct msp_activity_params {
  double a_exc, b_exc, c_exc, d_exc;
  double a_inh, b_inh, c_inh, d_inh;
  double w_exc, w_inh;
  double bg_mean, bg_width;
  double ca_beta, ca_tau;
  int32_t epoch;
} msp_activity_params;

/*
 * Initial state of the activity (Sec. II: the neuron model's state before the first
 * step): v = c and u = b c of the neuron's type (its reset potential and the resting
 * relation of the recovery variable), calcium = 0, spiked = 0, epoch_count = 0,
 * freq = 0, written to the caller's device arrays [n] (the same arrays as
 * msp_activity_run's). MSP_ERR_INVALID for n < 1, a null pointer, or a type > 1
 * (found on the device; such a neuron is initialised as inhibitory). Waits on `s`.
 */
msp_status msp_activity_init(int64_t n, const uint8_t* neuron_type,
                             const msp_activity_params* params, double* v, double* u,
                             double* calcium, uint8_t* spiked, int32_t* epoch_count, double* freq,
                             hipStream_t s);

/*
 * Runs steps t0 .. t0 + steps - 1 (1 ms each). Per step t:
 *   1. exchange: synapse s (syn_src -> syn_tgt, syn_type = the source's type 0/1)
 *      carries the spike its source recorded in step t - 1 (spiked). With approx = 1,
 *      the synapses whose two neurons have different `rank` (the processes of a
 *      distributed run) instead carry a spike iff u < freq[source], u = (word 0 >> 11)
 *      2^-53 of Philox4x64-10 with key (seed, 5) and counter (s, t, 0, 0); approx = 2
 *      does so for every synapse; approx = 0 exchanges every spike. Each target counts
 *      the excitatory (e) and inhibitory (h) spikes it receives;
 *   2. I = w_exc e - w_inh h + bg_mean + bg_width (u' - 1/2), u' as above with key
 *      (seed, 6) and counter (neuron, t, 0, 0); v += (0.04 v^2 + 5 v + 140 - u + I) / 2
 *      twice, then u += a (b v - u); v >= 30 is a spike: v = c, u += d, spiked = 1;
 *   3. calcium -= calcium / ca_tau, then += ca_beta on a spike;
 *   4. if (t + 1) % epoch == 0: freq = epoch_count / epoch (spikes per step), and
 *      epoch_count restarts at 0.
 * All state is device memory of the caller, updated in place: v, u, calcium, freq
 * [n] float64; spiked [n] uint8; epoch_count [n] int32. rank [n] int32 is needed for
 * approx = 1 only. last_input (nullable, [2][n] int32) receives e and h of the last
 * step; spikes (nullable device int64 scalar) is incremented by the spikes of the run.
 * Errors: MSP_ERR_INVALID for n < 1, m < 0, steps < 0, approx outside 0..2, a null
 * pointer that is needed, epoch < 1 or ca_tau <= 0; a synapse with an endpoint
 * outside [0, n) or a type > 1 is skipped and the call returns MSP_ERR_INVALID after
 * the run. Waits on `s` once, at the end.
 */
msp_status msp_activity_run(int64_t n, const uint8_t* neuron_type, const int32_t* rank,
                            int64_t m, const int32_t* syn_src, const int32_t* syn_tgt,
                            const uint8_t* syn_type, int32_t approx,
                            const msp_activity_params* params, uint64_t seed, uint64_t t0,
                            int32_t steps, double* v, double* u, double* calcium,
                            uint8_t* spiked, int32_t* epoch_count, double* freq,
                            int32_t* last_input, int64_t* spikes, hipStream_t s);

#ifdef __cplusplus
}
#endif

#endif /* MSP_H */
