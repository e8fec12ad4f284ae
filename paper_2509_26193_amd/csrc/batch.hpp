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

struct SimDesc {
  const NodeRec* rec[2];
  const int32_t* vs[2];
  const double* pos;
  const int32_t* order;
  const int32_t* nbeg;
  const int32_t* nend;
  const int32_t* leaf_of;
  int32_t* err;                 // the octree's sticky device flag
  const uint8_t* type;          // [n]
  const int32_t* vac_axon;      // [n]
  int64_t* elem_off;            // [n + 1] output
  int32_t* target;              // [capacity] output
  int64_t capacity;
  int64_t n;
  double L2, theta2, k2;
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
  int32_t* tile_base;           // [nsims + 1]
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
  A.type = d->type;
  A.vac_axon = d->vac_axon;
  A.elem_off = d->elem_off;
  A.work = work;
  A.target = d->target;
  A.err = d->err;
  A.L2 = d->L2;
  A.theta2 = d->theta2;
  A.k2 = d->k2;
  A.seed = d->seed;
  A.step = d->step;
  return A;
}

// Persistent waves pull 64-source tiles: first from the Morton range of their own
// die (neighbouring sources share upper-tree nodes in that die's L2), then from the
// other dies' ranges. A tile's simulation is found from the tile bases.
template <bool DIAG, int SLOTS>
__global__ void __launch_bounds__(kWaveBlock) search_sweep_k(BatchDev B, SweepOut W) {
  const int lane = threadIdx.x & (kWave - 1);
  const int home = blockIdx.x % kXcd;
  const int ntiles = *W.tile_count;
  int q = 0;
  int step0 = 2 * kCkptStepMin;
  while (q < kXcd) {
    const int qq = (home + q) % kXcd;
    const int lo = (int)((int64_t)ntiles * qq / kXcd);
    const int hi = (int)((int64_t)ntiles * (qq + 1) / kXcd);
    int got = 0;
    if (lane == 0) got = atomicAdd(&W.queue[qq], 1);
    got = __shfl(got, 0, kWave);
    if (lo + got >= hi) {
      ++q;
      continue;
    }
    const int tile = lo + got;
    const int sim = __builtin_amdgcn_readfirstlane(
        find_sim(as_const(B.tile_base), B.nsims, (int64_t)tile));
    const SearchArgs A = args_of(B.sims, sim, B.work);
    const int steps = sweep_tile<DIAG, SLOTS>(A, W, tile, lane, step0);
    if constexpr (SLOTS > 0) {
      // next interval: about SLOTS checkpoints over a sweep as long as this one
      step0 = kCkptStepMin;
      while (step0 * SLOTS < steps) step0 <<= 1;
    }
  }
}

// One thread per worklist slot (source): its elements' draws and restarts. The 64
// slots of a wavefront form one tile, so the simulation is uniform across the wave.
template <bool DIAG, int SLOTS>
__global__ void __launch_bounds__(256) search_draw_k(BatchDev B, SweepOut W) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tile = slot / kWave;
  if (tile >= *W.tile_count) return;
  const int sim = __builtin_amdgcn_readfirstlane(find_sim(as_const(B.tile_base), B.nsims, tile));
  const SearchArgs A = args_of(B.sims, sim, B.work);
  DiagOut D{};
  if (DIAG) {
    const cptr<SimDesc> d = as_const(B.sims) + sim;
    D.z0 = d->diag.z0;
    D.levels = d->diag.levels;
    D.visits = d->diag.visits;
    D.opens = d->diag.opens;
    D.visits0 = d->diag.visits0;
    D.opens0 = d->diag.opens0;
  }
  draw_slot<DIAG, SLOTS>(A, D, W, slot);
}

__global__ void fill_i32_k(int32_t* p, int64_t n, int32_t v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
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
    if ((inv || cap) && (int)(threadIdx.x & (kWave - 1)) == first)
      atomicOr(&B.status[s0], (inv ? kSimInvalid : 0) | (cap ? kSimCapacity : 0));
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

struct FlatSource {             // flat Morton position g is a type-`want` source
  BatchDev B;
  uint8_t want;
  __device__ int32_t operator()(int32_t, int64_t g) const {
    const int s = find_sim(B.nbase, B.nsims, g);
    if (B.status[s] != 0) return 0;
    const SimDesc& d = B.sims[s];
    const int32_t id = d.order[g - B.nbase[s]];
    return (d.vac_axon[id] > 0 && (d.type[id] ? 1 : 0) == want) ? 1 : 0;
  }
};

// Tiles per simulation: excitatory sources padded to a multiple of 64, then
// inhibitory ones, so no tile mixes simulations or types. One thread.
__global__ void b_tiles_k(BatchDev B, int32_t* tile_count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t t = 0;
  for (int s = 0; s < B.nsims; ++s) {
    B.tile_base[s] = t;
    const int64_t b = B.nbase[s], e = B.nbase[s + 1];
    const int32_t c0 = B.p0[e] - B.p0[b], c1 = B.p1[e] - B.p1[b];
    t += (c0 + kWave - 1) / kWave + (c1 + kWave - 1) / kWave;
  }
  B.tile_base[B.nsims] = t;
  *tile_count = t;
}

__global__ void b_work_k(BatchDev B, int64_t total) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int s = find_sim(B.nbase, B.nsims, g);
  if (B.status[s] != 0) return;
  const int64_t b = B.nbase[s], e = B.nbase[s + 1];
  const SimDesc& d = B.sims[s];
  const int32_t id = d.order[g - b];
  if (d.vac_axon[id] <= 0) return;
  const int64_t base = (int64_t)B.tile_base[s] * kWave;
  int64_t slot;
  if (d.type[id]) {
    const int32_t c0 = B.p0[e] - B.p0[b];
    slot = base + (int64_t)((c0 + kWave - 1) / kWave) * kWave + (B.p1[g] - B.p1[b]);
  } else {
    slot = base + (B.p0[g] - B.p0[b]);
  }
  B.work[slot] = id;
}

// ---------------------------------------------------------------------------
// Scratch layout (device), carved from one buffer.
// ---------------------------------------------------------------------------
struct SearchScratch {
  BatchDev B;
  SweepOut W;
  int32_t* counters;            // [0] tile count, [1..8] die queues
  void* scan_tmp;
};

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

inline int64_t max_tiles_for(int64_t total_n, int nsims) { return total_n / kWave + 2 * nsims + 1; }

struct ScratchSizes {
  size_t ea, p, tile_base, status, work, Z, v, nck, ckx, ckP, ckme, counters, scan, total;
};

// Checkpoint bytes per slot of a tile: the wave position and, per lane, the running
// sum and the mask end.
constexpr size_t kCkptSlotBytes = sizeof(int32_t) + kWave * (sizeof(double) + sizeof(int32_t));

// `slots` checkpoint slots per tile (0: no checkpoints, for launches without draws).
inline ScratchSizes scratch_sizes(int64_t total_n, int nsims, int slots) {
  ScratchSizes z;
  const int64_t mt = max_tiles_for(total_n, nsims);
  const int64_t ms = mt * kWave;
  z.ea = align_up(sizeof(int64_t) * (total_n + 1));
  z.p = align_up(sizeof(int32_t) * (total_n + 1));
  z.tile_base = align_up(sizeof(int32_t) * (nsims + 1));
  z.status = align_up(sizeof(int32_t) * nsims);
  z.work = align_up(sizeof(int32_t) * ms);
  z.Z = align_up(sizeof(double) * ms);
  z.v = align_up(sizeof(int32_t) * ms);
  z.nck = align_up(sizeof(int32_t) * mt);
  z.ckx = align_up(sizeof(int32_t) * mt * slots);
  z.ckP = align_up(sizeof(double) * mt * slots * kWave);
  z.ckme = align_up(sizeof(int32_t) * mt * slots * kWave);
  z.counters = align_up(sizeof(int32_t) * (1 + kXcd));
  z.scan = align_up(std::max(scan_tmp_bytes<int64_t>(total_n), scan_tmp_bytes<int32_t>(total_n)));
  z.total = z.ea + 2 * z.p + z.tile_base + z.status + z.work + z.Z + 2 * z.v + z.nck + z.ckx +
            z.ckP + z.ckme + z.counters + z.scan;
  return z;
}

inline SearchScratch carve(void* base, int64_t total_n, int nsims, int slots,
                           const SimDesc* d_sims, const int64_t* d_nbase) {
  const ScratchSizes z = scratch_sizes(total_n, nsims, slots);
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
  S.B.status = reinterpret_cast<int32_t*>(take(z.status));
  S.B.work = reinterpret_cast<int32_t*>(take(z.work));
  S.B.max_slots = max_tiles_for(total_n, nsims) * kWave;
  S.W.Z = reinterpret_cast<double*>(take(z.Z));
  S.W.v0 = reinterpret_cast<int32_t*>(take(z.v));
  S.W.o0 = reinterpret_cast<int32_t*>(take(z.v));
  S.W.nck = reinterpret_cast<int32_t*>(take(z.nck));
  S.W.ck_x = reinterpret_cast<int32_t*>(take(z.ckx));
  S.W.ck_P = reinterpret_cast<double*>(take(z.ckP));
  S.W.ck_me = reinterpret_cast<int32_t*>(take(z.ckme));
  S.W.ck_slots = slots;
  S.counters = reinterpret_cast<int32_t*>(take(z.counters));
  S.W.tile_count = S.counters;
  S.W.queue = S.counters + 1;
  S.W.wave_steps = nullptr;
  S.scan_tmp = take(z.scan);
  return S;
}

// Preparation: status, CSR offsets, worklists, tile bases. Kernels only.
inline hipError_t enqueue_prep(SearchScratch& S, int64_t total_n, hipStream_t s) {
  BatchDev& B = S.B;
  const unsigned g = grid_for(total_n, 256);
  fill_i32_k<<<grid_for(B.nsims, 256), 256, 0, s>>>(B.status, B.nsims, 0);
  fill_i32_k<<<grid_for(B.max_slots, 256), 256, 0, s>>>(B.work, B.max_slots, -1);
  fill_i32_k<<<1, 64, 0, s>>>(S.counters, 1 + kXcd, 0);
  b_check_k<<<g, 256, 0, s>>>(B, total_n);
  hipError_t e = exclusive_scan<int64_t, int32_t, FlatAxon>(nullptr, B.ea, total_n, FlatAxon{B},
                                                             true, s, S.scan_tmp);
  if (e != hipSuccess) return e;
  b_offsets_k<<<g, 256, 0, s>>>(B, total_n);
  e = exclusive_scan<int32_t, int32_t, FlatSource>(nullptr, B.p0, total_n, FlatSource{B, 0}, true, s,
                                                   S.scan_tmp);
  if (e != hipSuccess) return e;
  e = exclusive_scan<int32_t, int32_t, FlatSource>(nullptr, B.p1, total_n, FlatSource{B, 1}, true, s,
                                                   S.scan_tmp);
  if (e != hipSuccess) return e;
  b_tiles_k<<<1, 64, 0, s>>>(B, S.counters);
  b_work_k<<<g, 256, 0, s>>>(B, total_n);
  return hipGetLastError();
}

// The sweep and draw launches. `sweep_blocks` persistent blocks; the draw covers
// every possible slot (threads past the tile count return at once).
inline hipError_t enqueue_search(SearchScratch& S, bool diag, unsigned sweep_blocks,
                                 int draw_block, hipStream_t s, hipEvent_t mid = nullptr) {
  const unsigned draw_grid = grid_for(S.B.max_slots, draw_block);
  const bool big = S.W.ck_slots == kCkptMax;
  if (diag && big)
    search_sweep_k<true, kCkptMax><<<sweep_blocks, kWaveBlock, 0, s>>>(S.B, S.W);
  else if (diag)
    search_sweep_k<true, kCkptMin><<<sweep_blocks, kWaveBlock, 0, s>>>(S.B, S.W);
  else if (big)
    search_sweep_k<false, kCkptMax><<<sweep_blocks, kWaveBlock, 0, s>>>(S.B, S.W);
  else
    search_sweep_k<false, kCkptMin><<<sweep_blocks, kWaveBlock, 0, s>>>(S.B, S.W);
  if (mid) {
    hipError_t e = hipEventRecord(mid, s);
    if (e != hipSuccess) return e;
  }
  if (diag && big)
    search_draw_k<true, kCkptMax><<<draw_grid, draw_block, 0, s>>>(S.B, S.W);
  else if (diag)
    search_draw_k<true, kCkptMin><<<draw_grid, draw_block, 0, s>>>(S.B, S.W);
  else if (big)
    search_draw_k<false, kCkptMax><<<draw_grid, draw_block, 0, s>>>(S.B, S.W);
  else
    search_draw_k<false, kCkptMin><<<draw_grid, draw_block, 0, s>>>(S.B, S.W);
  return hipGetLastError();
}

}  // namespace msp
