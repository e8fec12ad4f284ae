// Search over a batch of independent simulations: one set of launches for all of
// them. A single simulation (the plain msp_find_targets) is the batch of one, so a
// simulation's results do not depend on the batch it runs in.
//
// Every simulation s has its own octree, sources, parameters and outputs, described
// by a SimDesc in a device table. Flat index spaces concatenate the simulations'
// neurons (neuron g of the batch = neuron g - nbase[s] of simulation s) and their
// 64-source tiles (tile t belongs to simulation s for tile_base[s] <= t <
// tile_base[s + 1]). Preparation (CSR offsets, Morton worklists) runs as flat
// kernels over the batch; the sweep's persistent waves pull tiles of any simulation.
// Nothing here allocates or synchronises: the scratch comes from the caller, so the
// whole sequence can be captured in a HIP graph and replayed.
#pragma once

#include <algorithm>

#include "scan.hpp"
#include "search_wave.hpp"

namespace msp {

// LDS bytes per thread of the kernels that run restart levels: a level's kept weights
// and ids (see restart_search).
constexpr size_t kRestartLds = kRestartKeep * (sizeof(double) + sizeof(uint32_t));

struct SimDesc {
  const NodeRec* rec[2];
  const int32_t* vs[2];
  const double* pos;
  const int32_t* order;
  const uint64_t* keys;         // [n] sorted Morton keys (position g: neuron order[g])
  const int32_t* nbeg;
  const int32_t* nend;
  const int32_t* leaf_of;
  int32_t own;                  // per-thread walks test for the source's own cell
  int32_t inside;               // the octree's positions lie inside its cube
  int32_t* err;                 // the octree's sticky device flag
  const uint8_t* type;          // [n]
  const int32_t* vac_axon;      // [n]
  int64_t* elem_off;            // [n + 1] output
  int32_t* target;              // [capacity] output
  int64_t capacity;
  int64_t n;
  double L2, theta2, acc_d2, k2;  // acc_d2: accept_bound(L2, theta2)
  uint64_t seed, step;
  DiagOut diag;                 // nullable outputs of counting launches
};

// per-simulation status bits (device), 0 = ok
constexpr int32_t kSimInvalid = 1;     // negative vac_axon or a type > 1
constexpr int32_t kSimCapacity = 2;    // more searches than target capacity

struct BatchDev {
  const SimDesc* sims;          // [nsims]
  int32_t nsims;
  const int64_t* nbase;         // [nsims + 1] flat neuron offsets
  int64_t* ea;                  // [total + 1] flat exclusive scan of vac_axon
  int32_t* p0;                  // [total + 1] flat scan: excitatory sources, Morton order
  int32_t* p1;                  // [total + 1] flat scan: inhibitory sources, Morton order
  uint8_t* src_type;            // [total] type of the source at flat position g, 2: none
  int32_t* tile_base;           // [nsims + 1]
  int32_t* unit_base;           // [nsims + 1] sweep units (a tile's parts) before each
  uint8_t* plog;                // [nsims] log2 of the parts per tile
  int32_t* status;              // [nsims]
  int32_t* work;                // [max_slots] source id per slot, -1 = padding
  int64_t max_slots;
};

// Largest s with base[s] <= g (base ascending, base[0] = 0).
template <class T>
__device__ __forceinline__ int find_sim(const T* base, int nsims, int64_t g) {
  int lo = 0, hi = nsims - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)base[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ SearchArgs args_of(const SimDesc* sims, int s, const int32_t* work) {
  const cptr<SimDesc> d = as_const(sims) + s;
  SearchArgs A;
  A.rec[0] = d->rec[0];
  A.rec[1] = d->rec[1];
  A.vs[0] = d->vs[0];
  A.vs[1] = d->vs[1];
  A.pos = d->pos;
  A.order = d->order;
  A.nbeg = d->nbeg;
  A.nend = d->nend;
  A.leaf_of = d->leaf_of;
  A.own = d->own != 0;
  A.type = d->type;
  A.vac_axon = d->vac_axon;
  A.elem_off = d->elem_off;
  A.work = work;
  A.target = d->target;
  A.err = d->err;
  A.L2 = d->L2;
  A.theta2 = d->theta2;
  A.acc_d2 = d->acc_d2;
  A.k2 = d->k2;
  A.seed = d->seed;
  A.step = d->step;
  return A;
}

// Persistent waves pull units (parts of 64-source tiles, in tile order): first from
// the Morton range of their own die (neighbouring sources share upper-tree nodes in
// that die's L2), then from the other dies' ranges. A unit's simulation is found from
// the unit bases.
// Scalar registers: on this chip a wave that needs more than 80 (the count the compiler
// reports, with VCC) leaves room for only 7 waves per SIMD, although the compiler and the
// occupancy query both count 8 (measured: 78 give 8 resident waves per SIMD, 82 give 7).
// The sweep hides record latency with resident waves, so it is held to 80; what does not
// fit is kept in vector-register lanes on the rare paths (bucket leaves, thinning).
template <bool DIAG, int SLOTS, bool OWN>
__global__ void __launch_bounds__(kWaveBlock) __attribute__((amdgpu_num_sgpr(80)))
search_sweep_k(BatchDev B, SweepOut W) {
  const int lane = threadIdx.x & (kWave - 1);
  const int home = blockIdx.x % kXcd;
  const int nunits = *W.unit_count;
  const bool own = nunits <= W.ck_units;
  int q = 0;
  int prev = 0;                          // wave steps of this wave's previous unit
  while (q < kXcd) {
    const int qq = (home + q) % kXcd;
    const int lo = (int)((int64_t)nunits * qq / kXcd);
    const int hi = (int)((int64_t)nunits * (qq + 1) / kXcd);
    int got = 0;
    if (lane == 0) got = atomicAdd(&W.queue[qq], 1);
    got = __shfl(got, 0, kWave);
    if (lo + got >= hi) {
      ++q;
      continue;
    }
    const int unit = lo + got;
    const int sim = __builtin_amdgcn_readfirstlane(
        find_sim(as_const(B.unit_base), B.nsims, (int64_t)unit));
    const int plog = __builtin_amdgcn_readfirstlane((int)as_const(B.plog)[sim]);
    const int local = unit - as_const(B.unit_base)[sim];
    const int tile = as_const(B.tile_base)[sim] + (local >> plog);
    const int part = local & ((1 << plog) - 1);
    const SearchArgs A = args_of(B.sims, sim, B.work);
    // checkpoint interval: about as many checkpoints as the part has slots over a
    // walk as long as the previous one
    int step0 = 2 * kCkptStepMin;
    if (SLOTS > 0 && prev > 0) {
      // as many checkpoints per tile as without parts: a unit with a region of its
      // own keeps the rest of its slots as headroom (no thinning in long parts)
      step0 = kCkptStepMin;
      while (step0 * (SLOTS >> plog) < prev) step0 <<= 1;
    }
    prev = sweep_tile<DIAG, SLOTS, OWN>(A, W, tile, part, plog, unit, own, lane, step0);
  }
}

// One thread per worklist slot (source): its elements' draws and restarts. The 64
// slots of a wavefront form one tile, so the simulation is uniform across the wave.
template <bool DIAG, int SLOTS, bool DEFER>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) search_draw_k(BatchDev B, SweepOut W) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tile = slot / kWave;
  if (tile >= *W.tile_count) return;
  const int sim = __builtin_amdgcn_readfirstlane(find_sim(as_const(B.tile_base), B.nsims, tile));
  const SearchArgs A = args_of(B.sims, sim, B.work);
  const int plog = __builtin_amdgcn_readfirstlane((int)as_const(B.plog)[sim]);
  const int64_t u0 = (int64_t)as_const(B.unit_base)[sim] +
                     ((tile - (int64_t)as_const(B.tile_base)[sim]) << plog);
  DiagOut D{};
  if (DIAG) {
    const cptr<SimDesc> d = as_const(B.sims) + sim;
    D.z0 = d->diag.z0;
    D.levels = d->diag.levels;
    D.visits = d->diag.visits;
    D.opens = d->diag.opens;
    D.visits0 = d->diag.visits0;
    D.opens0 = d->diag.opens0;
    D.entries0 = d->diag.entries0;
  }
  // the restart levels' entries: kRestartKeep weights, then as many ids, per thread,
  // in LDS sized by the launch (kRestartLds bytes per thread)
  extern __shared__ double keep_lds[];
  const KeptEntries keep{keep_lds + threadIdx.x,
                         reinterpret_cast<uint32_t*>(keep_lds + kRestartKeep * blockDim.x) +
                             threadIdx.x,
                         (int)blockDim.x};
  draw_slot<DIAG, SLOTS, DEFER>(A, D, W, slot, u0, plog, *W.unit_count <= W.ck_units, &keep);
}

// Second phase of a two-phase search (one simulation): one thread per request in
// cell order (keys sorted); each continues its search from the deferred cell with the
// same draws as the one-phase search, so the target is the same.
template <bool DIAG>
__global__ void __launch_bounds__(256) search_phase2_k(BatchDev B, SweepOut W, int64_t nreq) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nreq) return;
  const uint64_t key = W.defer.key[q];
  if (key == W.defer.none) return;              // sorted last: no request from here on
  const int64_t e = W.defer.val[q];
  const SearchArgs A = args_of(B.sims, 0, B.work);
  const int32_t i = W.defer.src[e];
  const int32_t j = W.defer.elem[e];
  const int t = A.type[i] ? 1 : 0;
  const NodeRec* __restrict__ R = A.rec[t];
  const int32_t li = A.leaf_of[i];
  const double xi = A.pos[3 * (int64_t)i], yi = A.pos[3 * (int64_t)i + 1],
               zi = A.pos[3 * (int64_t)i + 2];
  int lev = W.defer.level[e];
  Count c;
  DiagOut D{};
  if (DIAG) {
    const cptr<SimDesc> d = as_const(B.sims);
    D.levels = d->diag.levels;
    D.visits = d->diag.visits;
    D.opens = d->diag.opens;
    if (D.visits) c.visits = D.visits[e];
    if (D.opens) c.opens = D.opens[e];
  }
  int32_t none = -1;
  extern __shared__ double keep_lds[];      // kRestartLds bytes per thread (see search_draw_k)
  const KeptEntries keep{keep_lds + threadIdx.x,
                         reinterpret_cast<uint32_t*>(keep_lds + kRestartKeep * blockDim.x) +
                             threadIdx.x,
                         (int)blockDim.x};
  const int32_t tgt = restart_search<DIAG, false>(A, R, A.vs[t], W.defer.cell[e], lev, kNoDefer,
                                                  i, j, li, xi, yi, zi, &lev, c, &none, &keep);
  A.target[e] = tgt;
  if (DIAG) {
    if (D.levels) D.levels[e] = lev;
    if (D.visits) D.visits[e] = c.visits;
    if (D.opens) D.opens[e] = c.opens;
  }
}

// Number of requests: the first position whose sorted key is `none`.
__global__ void phase2_count_k(SweepOut W, int64_t nreq, int64_t* out) {
  int64_t lo = 0, hi = nreq;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (W.defer.key[mid] == W.defer.none) hi = mid; else lo = mid + 1;
  }
  *out = lo;
}

// Validity of vac_axon and types; per-simulation status starts at 0 (fill before).
__global__ void b_check_k(BatchDev B, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int s = find_sim(B.nbase, B.nsims, g);
  const int64_t i = g - B.nbase[s];
  const SimDesc& d = B.sims[s];
  const int32_t a = d.vac_axon[i];
  int32_t f = (a < 0 || d.type[i] > 1) ? kSimInvalid : 0;
  if (a > 0 && d.target == nullptr) f |= kSimCapacity;
  // one atomic per wave and flag where the wave's lanes share a simulation (the
  // usual case); a wave that straddles two simulations reports lane by lane
  const int s0 = __builtin_amdgcn_readfirstlane(s);
  if (__all(s == s0)) {
    const bool inv = __ballot((f & kSimInvalid) != 0) != 0;
    const bool cap = __ballot((f & kSimCapacity) != 0) != 0;
    const int first = __ffsll((unsigned long long)__ballot(1)) - 1;
    const int32_t want = (inv ? kSimInvalid : 0) | (cap ? kSimCapacity : 0);
    // most waves of a failing simulation find the flags already set: no atomic then
    if (want && (int)(threadIdx.x & (kWave - 1)) == first &&
        (__hip_atomic_load(&B.status[s0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & want) !=
            want)
      atomicOr(&B.status[s0], want);
  } else if (f) {
    atomicOr(&B.status[s], f);
  }
}

struct FlatAxon {               // vac_axon of flat neuron g (by id), clamped at 0
  BatchDev B;
  __device__ int64_t operator()(int32_t, int64_t g) const {
    const int s = find_sim(B.nbase, B.nsims, g);
    const int32_t a = B.sims[s].vac_axon[g - B.nbase[s]];
    return a > 0 ? (int64_t)a : 0;
  }
};

// Per-simulation CSR offsets and the capacity check.
__global__ void b_offsets_k(BatchDev B, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int s = find_sim(B.nbase, B.nsims, g);
  const int64_t b = B.nbase[s], e = B.nbase[s + 1];
  const SimDesc& d = B.sims[s];
  d.elem_off[g - b] = B.ea[g] - B.ea[b];
  if (g == e - 1) {
    const int64_t S = B.ea[e] - B.ea[b];
    d.elem_off[e - b] = S;
    if (S > d.capacity) atomicOr(&B.status[s], kSimCapacity);
  }
}

// src_type[g]: the type (0, 1) of the neuron at flat Morton position g if it is a
// source of a simulation without errors, else 2. One gather per neuron; the scans and
// the worklist then read it in order.
__global__ void b_src_type_k(BatchDev B, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int s = find_sim(B.nbase, B.nsims, g);
  uint8_t st = 2;
  if (B.status[s] == 0) {
    const SimDesc& d = B.sims[s];
    const int32_t id = d.order[g - B.nbase[s]];
    if (d.vac_axon[id] > 0) st = d.type[id] ? 1 : 0;
  }
  B.src_type[g] = st;
}

struct FlatSource {             // flat Morton position g is a type-`want` source
  const uint8_t* src_type;
  uint8_t want;
  __device__ int32_t operator()(int32_t, int64_t g) const { return src_type[g] == want ? 1 : 0; }
};

// Tiles per simulation: excitatory sources padded to a multiple of 64, then
// inhibitory ones, so no tile mixes simulations or types. A simulation with few tiles
// cuts each into 2^p parts (p <= kPartLogMax): as many as keep its units within
// kPartUnits and, for a launch with checkpoints, within one checkpoint region per 64 of
// its neurons (every launch has at least that many); else 2 parts where that stays
// within 2 kPartUnits (a launch has up to twice those regions where memory allows, else
// the two parts share their tile's region). p depends on the simulation alone, so a
// simulation's results do not depend on the batch it runs in (force >= 0: p = force).
// One thread. Also writes the unit count and the number of sources (the length of the
// Hilbert sort).
__global__ void b_tiles_k(BatchDev B, int32_t* tile_count, int32_t* unit_count,
                          int32_t* sources, int64_t total, int force, bool ckpt) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t t = 0, u = 0;
  for (int s = 0; s < B.nsims; ++s) {
    B.tile_base[s] = t;
    B.unit_base[s] = u;
    const int64_t b = B.nbase[s], e = B.nbase[s + 1];
    const int32_t c0 = B.p0[e] - B.p0[b], c1 = B.p1[e] - B.p1[b];
    const int32_t ts = (c0 + kWave - 1) / kWave + (c1 + kWave - 1) / kWave;
    int p = force;
    if (p < 0) {
      const int64_t regions = (e - b) / kWave + 2;
      const int64_t lim = ckpt && regions < kPartUnits ? regions : kPartUnits;
      p = 0;
      while (p < kPartLogMax && ((int64_t)ts << (p + 1)) <= lim) ++p;
      if (p == 0 && 2 * (int64_t)ts <= 2 * (int64_t)kPartUnits) p = 1;
    }
    B.plog[s] = (uint8_t)p;
    t += ts;
    u += ts << p;
  }
  B.tile_base[B.nsims] = t;
  B.unit_base[B.nsims] = u;
  *tile_count = t;
  *unit_count = u;
  *sources = B.p0[total] + B.p1[total];
}

// Hilbert index of a cell of the 2^21 grid (J. Skilling, "Programming the Hilbert
// curve", AIP Conf. Proc. 707, 2004: axes to transposed index, then bit interleave).
// Only the order it induces matters here: sources consecutive along the curve are
// close in space, with none of the long jumps the Morton order makes between octants.
__device__ __forceinline__ uint64_t hilbert3(uint32_t x0, uint32_t x1, uint32_t x2) {
  uint32_t X[3] = {x0, x1, x2};
  for (uint32_t Q = 1u << 20; Q > 1; Q >>= 1) {
    const uint32_t P = Q - 1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;                                  // invert
      } else {
        const uint32_t t = (X[0] ^ X[i]) & P;       // exchange
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0;
  for (uint32_t Q = 1u << 20; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  X[0] ^= t;
  X[1] ^= t;
  X[2] ^= t;
  uint64_t h = 0;
  for (int b = 20; b >= 0; --b)
    h = (h << 3) | ((uint64_t)((X[0] >> b) & 1u) << 2) | ((uint64_t)((X[1] >> b) & 1u) << 1) |
        (uint64_t)((X[2] >> b) & 1u);
  return h;
}

// The three 21-bit cell coordinates of a Morton key (digit 4x + 2y + z per level).
__device__ __forceinline__ void morton_decode(uint64_t k, uint32_t& x, uint32_t& y, uint32_t& z) {
  x = y = z = 0;
  for (int b = 20; b >= 0; --b) {
    const uint32_t d = (uint32_t)(k >> (3 * b)) & 7u;
    x = (x << 1) | (d >> 2);
    y = (y << 1) | ((d >> 1) & 1u);
    z = (z << 1) | (d & 1u);
  }
}

// Sort keys of the sources: (simulation, type) group in the top `gb` of `kb` bits, then
// the leading kb - gb bits of the Hilbert index; value = flat Morton position. Sources
// are packed in Morton order (position p0 + p1), so only that prefix is sorted.
__global__ void b_hkeys_k(BatchDev B, int64_t total, int gb, int kb, uint64_t* key,
                          int32_t* val) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int t = B.src_type[g];
  if (t > 1) return;
  const int s = find_sim(B.nbase, B.nsims, g);
  const SimDesc& d = B.sims[s];
  uint32_t x, y, z;
  morton_decode(d.keys[g - B.nbase[s]], x, y, z);
  const int hb = kb - gb;
  const uint64_t h = hilbert3(x, y, z) >> (63 - hb);
  const int64_t idx = (int64_t)B.p0[g] + B.p1[g];
  key[idx] = ((uint64_t)(2 * s + t) << hb) | h;
  val[idx] = (int32_t)g;
}

// Worklist from the sorted sources: the rank within a (simulation, type) group is the
// sorted position minus the group's start.
__global__ void b_work_sorted_k(BatchDev B, int64_t total, const int32_t* __restrict__ val) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)B.p0[total] + B.p1[total]) return;
  const int64_t g = val[p];
  const int s = find_sim(B.nbase, B.nsims, g);
  const int64_t b = B.nbase[s], e = B.nbase[s + 1];
  const SimDesc& d = B.sims[s];
  const int32_t id = d.order[g - b];
  const int t = B.src_type[g];
  const int32_t c0 = B.p0[e] - B.p0[b];
  const int64_t start = (int64_t)B.p0[b] + B.p1[b] + (t ? c0 : 0);
  const int64_t base = (int64_t)B.tile_base[s] * kWave +
                       (t ? (int64_t)((c0 + kWave - 1) / kWave) * kWave : 0);
  B.work[base + (p - start)] = id;
}

// ---------------------------------------------------------------------------
// Scratch layout (device), carved from one buffer.
// ---------------------------------------------------------------------------
struct SearchScratch {
  BatchDev B;
  SweepOut W;
  int32_t* counters;            // [0] tile count, [1..8] die queues, [9] sources, [10] units
  void* scan_tmp;
  uint64_t* hkey[2];            // [total_n] sort keys of the Hilbert-ordered worklist
  int32_t* hval[2];             // [total_n] their flat positions
  void* hsort;                  // radix sort workspace
  bool own_cell;                // the sweep tests for the source's own cell (see sweep_tile)
};

inline int64_t max_tiles_for(int64_t total_n, int nsims) { return total_n / kWave + 2 * nsims + 1; }

// Sweep units: a simulation has at most 2^kPartLogMax units per tile, and more units
// than tiles only while they stay within kPartUnits or, with 2 parts, while its tiles do;
// with the parts forced to 2^force (force >= 0), exactly that many per tile.
inline int64_t max_units_for(int64_t total_n, int nsims, int force = -1) {
  const int64_t mt = max_tiles_for(total_n, nsims);
  if (force >= 0) return mt << force;
  return std::min(mt << kPartLogMax, mt + (int64_t)nsims * kPartUnits);
}

struct ScratchSizes {
  size_t ea, p, tile_base, unit_base, plog, status, work, Z, v, nck, ckx, ckP, ckme, counters,
      scan, srct, hkey, hval, hsort, total;
};

// Checkpoint bytes per slot of a tile: the wave position and, per lane, the running
// sum and the mask end.
constexpr size_t kCkptSlotBytes = sizeof(int32_t) + kWave * (sizeof(double) + sizeof(int32_t));

// `slots` checkpoint slots per tile (0: no checkpoints, for launches without draws).
// regions: checkpoint regions of `slots` slots (< 0: one per tile).
inline ScratchSizes scratch_sizes(int64_t total_n, int nsims, int slots, int force = -1,
                                  int64_t regions = -1) {
  ScratchSizes z;
  const int64_t mt = max_tiles_for(total_n, nsims);
  const int64_t ms = mt * kWave;
  const int64_t mu = max_units_for(total_n, nsims, force);
  z.ea = align_up(sizeof(int64_t) * (total_n + 1));
  z.p = align_up(sizeof(int32_t) * (total_n + 1));
  z.tile_base = align_up(sizeof(int32_t) * (nsims + 1));
  z.unit_base = align_up(sizeof(int32_t) * (nsims + 1));
  z.plog = align_up(sizeof(uint8_t) * nsims);
  z.status = align_up(sizeof(int32_t) * nsims);
  z.work = align_up(sizeof(int32_t) * ms);
  z.Z = align_up(sizeof(double) * mu * kWave);
  z.v = align_up(sizeof(int32_t) * mu * kWave);
  z.nck = align_up(sizeof(int32_t) * mu);
  const int64_t mr = regions < 0 ? mt : regions;
  z.ckx = align_up(sizeof(int32_t) * mr * slots);
  z.ckP = align_up(sizeof(double) * mr * slots * kWave);
  z.ckme = align_up(sizeof(int32_t) * mr * slots * kWave);
  z.counters = align_up(sizeof(int32_t) * (3 + kXcd));
  z.scan = align_up(std::max(scan_tmp_bytes<int64_t>(total_n), scan_tmp_bytes<int32_t>(total_n)));
  z.srct = align_up(sizeof(uint8_t) * total_n);
  z.hkey = align_up(sizeof(uint64_t) * total_n);
  z.hval = align_up(sizeof(int32_t) * total_n);
  z.hsort = align_up(radix_sort_ws_bytes(total_n));
  z.total = z.ea + 2 * z.p + z.tile_base + z.unit_base + z.plog + z.status + z.work + z.Z +
            3 * z.v + z.nck + z.ckx +
            z.ckP + z.ckme + z.counters + z.scan + z.srct + 2 * z.hkey + 2 * z.hval + z.hsort;
  return z;
}

inline SearchScratch carve(void* base, int64_t total_n, int nsims, int slots,
                           const SimDesc* d_sims, const int64_t* d_nbase, int force = -1,
                           int64_t regions = -1) {
  const ScratchSizes z = scratch_sizes(total_n, nsims, slots, force, regions);
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += bytes;
    return q;
  };
  SearchScratch S{};
  S.B.sims = d_sims;
  S.B.nsims = nsims;
  S.B.nbase = d_nbase;
  S.B.ea = reinterpret_cast<int64_t*>(take(z.ea));
  S.B.p0 = reinterpret_cast<int32_t*>(take(z.p));
  S.B.p1 = reinterpret_cast<int32_t*>(take(z.p));
  S.B.tile_base = reinterpret_cast<int32_t*>(take(z.tile_base));
  S.B.unit_base = reinterpret_cast<int32_t*>(take(z.unit_base));
  S.B.plog = reinterpret_cast<uint8_t*>(take(z.plog));
  S.B.status = reinterpret_cast<int32_t*>(take(z.status));
  S.B.work = reinterpret_cast<int32_t*>(take(z.work));
  S.B.max_slots = max_tiles_for(total_n, nsims) * kWave;
  S.W.Z = reinterpret_cast<double*>(take(z.Z));
  S.W.v0 = reinterpret_cast<int32_t*>(take(z.v));
  S.W.o0 = reinterpret_cast<int32_t*>(take(z.v));
  S.W.e0 = reinterpret_cast<int32_t*>(take(z.v));
  S.W.nck = reinterpret_cast<int32_t*>(take(z.nck));
  S.W.ck_x = reinterpret_cast<int32_t*>(take(z.ckx));
  S.W.ck_P = reinterpret_cast<double*>(take(z.ckP));
  S.W.ck_me = reinterpret_cast<int32_t*>(take(z.ckme));
  S.W.ck_slots = slots;
  S.W.ck_units = regions < 0 ? max_tiles_for(total_n, nsims) : regions;
  S.counters = reinterpret_cast<int32_t*>(take(z.counters));
  S.W.tile_count = S.counters;
  S.W.unit_count = S.counters + 2 + kXcd;
  S.W.queue = S.counters + 1;
  S.W.wave_steps = nullptr;
  S.own_cell = true;
  S.scan_tmp = take(z.scan);
  S.B.src_type = reinterpret_cast<uint8_t*>(take(z.srct));
  S.hkey[0] = reinterpret_cast<uint64_t*>(take(z.hkey));
  S.hkey[1] = reinterpret_cast<uint64_t*>(take(z.hkey));
  S.hval[0] = reinterpret_cast<int32_t*>(take(z.hval));
  S.hval[1] = reinterpret_cast<int32_t*>(take(z.hval));
  S.hsort = take(z.hsort);
  return S;
}

// Preparation: status, CSR offsets, worklists, tile and unit bases. Kernels only.
// force >= 0: every tile has 2^force parts (the scratch carved for it). ckpt: the
// sweep will write checkpoints.
inline hipError_t enqueue_prep(SearchScratch& S, int64_t total_n, hipStream_t s, int force = -1,
                               bool ckpt = true) {
  BatchDev& B = S.B;
  const unsigned g = grid_for(total_n, 256);
  fill_i32_k<<<grid_for(B.nsims, 256), 256, 0, s>>>(B.status, B.nsims, 0);
  fill_i32_k<<<grid_for(B.max_slots, 256), 256, 0, s>>>(B.work, B.max_slots, -1);
  fill_i32_k<<<1, 64, 0, s>>>(S.counters, 3 + kXcd, 0);
  b_check_k<<<g, 256, 0, s>>>(B, total_n);
  hipError_t e = exclusive_scan<int64_t, int32_t, FlatAxon>(nullptr, B.ea, total_n, FlatAxon{B},
                                                             true, s, S.scan_tmp);
  if (e != hipSuccess) return e;
  b_offsets_k<<<g, 256, 0, s>>>(B, total_n);
  b_src_type_k<<<g, 256, 0, s>>>(B, total_n);
  e = exclusive_scan<int32_t, int32_t, FlatSource>(nullptr, B.p0, total_n,
                                                   FlatSource{B.src_type, 0}, true, s, S.scan_tmp);
  if (e != hipSuccess) return e;
  e = exclusive_scan<int32_t, int32_t, FlatSource>(nullptr, B.p1, total_n,
                                                   FlatSource{B.src_type, 1}, true, s, S.scan_tmp);
  if (e != hipSuccess) return e;
  b_tiles_k<<<1, 64, 0, s>>>(B, S.counters, S.counters + 2 + kXcd, S.counters + 1 + kXcd,
                             total_n, force, ckpt);
  // 64-source tiles in Hilbert order within each (simulation, type) group
  // (32-bit keys keep 20 or more Hilbert bits, cells of about a hundredth of the box
  // edge or finer, for up to 2048 simulations)
  int gb = 1;
  while ((1ll << gb) < 2ll * B.nsims) ++gb;
  const int kb = gb <= 12 ? 32 : 48;
  b_hkeys_k<<<g, 256, 0, s>>>(B, total_n, gb, kb, S.hkey[0], S.hval[0]);
  e = radix_sort_pairs_ws(S.hkey[0], S.hval[0], S.hkey[1], S.hval[1], total_n, kb, s, S.hsort,
                          S.counters + 1 + kXcd);
  if (e != hipSuccess) return e;
  b_work_sorted_k<<<g, 256, 0, s>>>(B, total_n, S.hval[0]);
  return hipGetLastError();
}

// The sweep and draw launches. `sweep_blocks` persistent blocks; the draw covers
// every possible slot (threads past the tile count return at once).
template <bool DIAG, int SLOTS>
inline void launch_sweep(const SearchScratch& S, unsigned blocks, hipStream_t s) {
  if (S.own_cell)
    search_sweep_k<DIAG, SLOTS, true><<<blocks, kWaveBlock, 0, s>>>(S.B, S.W);
  else
    search_sweep_k<DIAG, SLOTS, false><<<blocks, kWaveBlock, 0, s>>>(S.B, S.W);
}

template <bool DIAG, int SLOTS>
inline void launch_draw(const SearchScratch& S, unsigned grid, int block, hipStream_t s) {
  if (S.W.defer.depth < kNoDefer)
    search_draw_k<DIAG, SLOTS, true><<<grid, block, kRestartLds * block, s>>>(S.B, S.W);
  else
    search_draw_k<DIAG, SLOTS, false><<<grid, block, kRestartLds * block, s>>>(S.B, S.W);
}

inline hipError_t enqueue_search(SearchScratch& S, bool diag, unsigned sweep_blocks,
                                 int draw_block, hipStream_t s, hipEvent_t mid = nullptr) {
  const unsigned draw_grid = grid_for(S.B.max_slots, draw_block);
  const bool big = S.W.ck_slots == kCkptMax;
  if (diag && big)
    launch_sweep<true, kCkptMax>(S, sweep_blocks, s);
  else if (diag)
    launch_sweep<true, kCkptMin>(S, sweep_blocks, s);
  else if (big)
    launch_sweep<false, kCkptMax>(S, sweep_blocks, s);
  else
    launch_sweep<false, kCkptMin>(S, sweep_blocks, s);
  if (mid) {
    hipError_t e = hipEventRecord(mid, s);
    if (e != hipSuccess) return e;
  }
  if (diag && big)
    launch_draw<true, kCkptMax>(S, draw_grid, draw_block, s);
  else if (diag)
    launch_draw<true, kCkptMin>(S, draw_grid, draw_block, s);
  else if (big)
    launch_draw<false, kCkptMax>(S, draw_grid, draw_block, s);
  else
    launch_draw<false, kCkptMin>(S, draw_grid, draw_block, s);
  return hipGetLastError();
}

}  // namespace msp
