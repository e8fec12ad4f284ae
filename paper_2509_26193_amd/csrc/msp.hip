// libmsp: C ABI entry points (declared in include/msp.h). One translation unit.
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <new>

#include "common.hpp"
#include "scan.hpp"
#include "build.hpp"
#include "refresh.hpp"
#include "search.hpp"
#include "search_wave.hpp"
#include "commit.hpp"

using namespace msp;

namespace {

template <class T>
hipError_t dalloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  return hipMalloc((void**)p, sizeof(T) * (size_t)count);
}

void release(msp_octree_s* t) {
  if (!t) return;
  void* ptrs[] = {t->pos, t->keys, t->order, t->leaf_of, t->skip, t->depth, t->nbeg, t->nend,
                  t->level_nodes, t->rec[0], t->rec[1], t->err};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (t->vs[0]) (void)hipFree(t->vs[0]);
  if (t->vs[1]) (void)hipFree(t->vs[1]);
  t->magic = kDead;
  delete t;
}

struct CountPos {
  __device__ int64_t operator()(int32_t a, int64_t) const { return a > 0 ? (int64_t)a : 0; }
};

struct SrcFlag {
  const int32_t* a;
  const uint8_t* ty;
  uint8_t want;
  __device__ int32_t operator()(int32_t id, int64_t) const {
    return (a[id] > 0 && (ty[id] ? 1 : 0) == want) ? 1 : 0;
  }
};

struct AccFlag {
  __device__ int64_t operator()(uint8_t a, int64_t) const { return (int64_t)a; }
};

__global__ void check_axon_k(const int32_t* __restrict__ a, const uint8_t* __restrict__ ty,
                             int64_t n, int32_t* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (a[i] < 0 || ty[i] > 1) atomicOr(flag, 1);
}

// Sources with a_i > 0 in Morton order: excitatory ones first, then inhibitory ones
// from the next multiple of 64, so that no 64-source tile mixes the two types.
// Unused slots hold -1. count[0] = number of tiles.
__global__ void worklist_k(const int32_t* __restrict__ order, const int32_t* __restrict__ a,
                           const uint8_t* __restrict__ ty, int64_t n,
                           const int32_t* __restrict__ p0, const int32_t* __restrict__ p1,
                           int32_t* __restrict__ work, int32_t* __restrict__ count) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t base1 = (p0[n] + kWave - 1) / kWave * kWave;
  if (m == 0) *count = (base1 + (p1[n] + kWave - 1) / kWave * kWave) / kWave;
  if (m >= n) return;
  const int32_t id = order[m];
  if (a[id] <= 0) return;
  if (ty[id]) work[base1 + p1[m]] = id;
  else work[p0[m]] = id;
}

// One thread per worklist slot (the first, per-source kernel).
__global__ void tiles_to_slots_k(const int32_t* __restrict__ tiles, int32_t* __restrict__ slots) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *slots = *tiles * kWave;
}

bool use_simple_kernel() {
  const char* e = getenv("MSP_SEARCH_KERNEL");
  return e && std::strcmp(e, "simple") == 0;
}

}  // namespace

extern "C" {

const char* msp_status_string(msp_status st) {
  switch (st) {
    case MSP_OK: return "ok";
    case MSP_ERR_INVALID: return "invalid argument or handle";
    case MSP_ERR_OOM: return "device out of memory";
    case MSP_ERR_HIP: return "HIP runtime error";
    case MSP_ERR_CAPACITY: return "output capacity exceeded";
    case MSP_ERR_DEVICE: return "data error detected on the device";
    case MSP_ERR_UNIMPLEMENTED: return "not implemented";
    default: return "unknown status";
  }
}

msp_status msp_sync(hipStream_t s) {
  MSP_HIP_TRY(hipStreamSynchronize(s));
  return MSP_OK;
}

msp_status msp_build_octree(const double* pos, int64_t n, const double box_min[3],
                            double box_edge, int32_t leaf_size, hipStream_t s, msp_octree* out) {
  if (!out) return MSP_ERR_INVALID;
  *out = nullptr;
  if (!pos || !box_min || n < 1 || n > MSP_MAX_NEURONS || leaf_size != 1) return MSP_ERR_INVALID;
  if (!std::isfinite(box_edge) || !(box_edge > 0.0)) return MSP_ERR_INVALID;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(box_min[a])) return MSP_ERR_INVALID;

  msp_octree_s* t = new (std::nothrow) msp_octree_s();
  if (!t) return MSP_ERR_OOM;
  std::memset(t, 0, sizeof(*t));
  t->magic = kMagic;
  t->n = n;
  t->box_edge = box_edge;
  for (int a = 0; a < 3; ++a) t->box_min[a] = box_min[a];
  if (hipGetDevice(&t->device) != hipSuccess) { release(t); return MSP_ERR_HIP; }

#define TRY(expr)                                               \
  do {                                                          \
    hipError_t e_ = (expr);                                     \
    if (e_ != hipSuccess) {                                     \
      (void)hipGetLastError();                                  \
      (void)hipStreamSynchronize(s);                            \
      release(t);                                               \
      return e_ == hipErrorOutOfMemory ? MSP_ERR_OOM : MSP_ERR_HIP; \
    }                                                           \
  } while (0)

  TRY(dalloc(&t->pos, 3 * n));
  TRY(dalloc(&t->keys, n));
  TRY(dalloc(&t->order, n));
  TRY(dalloc(&t->leaf_of, n));
  TRY(dalloc(&t->err, 1));
  TRY(dalloc(&t->vs[0], n));
  TRY(dalloc(&t->vs[1], n));
  TRY(hipMemsetAsync(t->err, 0, sizeof(int32_t), s));
  {
    Temp k1(s), v1(s), cnt(s), base(s), lvl(s);
    TRY(k1.alloc(sizeof(uint64_t) * n));
    TRY(v1.alloc(sizeof(int32_t) * n));
    keys_k<<<grid_for(n, kBuildBlock), kBuildBlock, 0, s>>>(pos, n, box_min[0], box_min[1],
                                                            box_min[2], box_edge, t->pos, t->keys,
                                                            t->order, t->err);
    TRY(hipGetLastError());
    TRY(radix_sort_pairs(t->keys, t->order, k1.as<uint64_t>(), v1.as<int32_t>(), n, 63, s));
    TRY(cnt.alloc(sizeof(int32_t) * n));
    TRY(base.alloc(sizeof(int32_t) * (n + 1)));
    node_count_k<<<grid_for(n, kBuildBlock), kBuildBlock, 0, s>>>(t->keys, n, cnt.as<int32_t>());
    TRY(hipGetLastError());
    TRY((exclusive_scan<int32_t, int32_t, Ident<int32_t>>(cnt.as<int32_t>(), base.as<int32_t>(), n,
                                                          Ident<int32_t>(), true, s)));
    int32_t N32 = 0;
    TRY(hipMemcpyAsync(&N32, base.as<int32_t>() + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    if (N32 < 1 || N32 >= kMaxNodes) {
      release(t);
      return MSP_ERR_INVALID;
    }
    const int64_t N = N32;
    t->N = N;
    TRY(dalloc(&t->skip, N));
    TRY(dalloc(&t->depth, N));
    TRY(dalloc(&t->nbeg, N));
    TRY(dalloc(&t->nend, N));
    TRY(dalloc(&t->level_nodes, N));
    TRY(dalloc(&t->rec[0], N + 1));           // + a sentinel record at index N
    TRY(dalloc(&t->rec[1], N + 1));
    TRY(hipMemsetAsync(t->rec[0] + N, 0, sizeof(NodeRec), s));
    TRY(hipMemsetAsync(t->rec[1] + N, 0, sizeof(NodeRec), s));
    TRY(lvl.alloc(sizeof(int32_t) * 2 * (kMaxDepth + 1)));
    int32_t* lcnt = lvl.as<int32_t>();
    TRY(hipMemsetAsync(lcnt, 0, sizeof(int32_t) * 2 * (kMaxDepth + 1), s));
    nodes_k<<<grid_for(n, kBuildBlock), kBuildBlock, 0, s>>>(t->keys, t->order, n,
                                                             base.as<int32_t>(), t->skip, t->depth,
                                                             t->nbeg, t->nend, t->leaf_of);
    TRY(hipGetLastError());
    level_count_k<<<grid_for(N, kBuildBlock), kBuildBlock, 0, s>>>(t->depth, N, lcnt);
    TRY(hipGetLastError());
    int32_t hc[kMaxDepth + 1];
    TRY(hipMemcpyAsync(hc, lcnt, sizeof(hc), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    int32_t hoff[kMaxDepth + 1];
    t->level_off[0] = 0;
    for (int k = 0; k <= kMaxDepth; ++k) {
      hoff[k] = (int32_t)t->level_off[k];
      t->level_off[k + 1] = t->level_off[k] + hc[k];
    }
    if (t->level_off[kMaxDepth + 1] != N) {
      release(t);
      return MSP_ERR_HIP;
    }
    int32_t* cursor = lcnt + (kMaxDepth + 1);
    TRY(hipMemcpyAsync(cursor, hoff, sizeof(hoff), hipMemcpyHostToDevice, s));
    level_scatter_k<<<grid_for(N, kBuildBlock), kBuildBlock, 0, s>>>(t->depth, N, cursor,
                                                                     t->level_nodes);
    TRY(hipGetLastError());
    init_meta_k<<<grid_for(N, kBuildBlock), kBuildBlock, 0, s>>>(t->skip, t->depth, t->nbeg,
                                                                 t->nend, t->order, N, t->rec[0],
                                                                 t->rec[1]);
    TRY(hipGetLastError());
    // the temporaries are released on `s`; make sure `hoff` (host) was consumed
    TRY(hipStreamSynchronize(s));
  }
#undef TRY
  *out = t;
  return MSP_OK;
}

void msp_free_octree(msp_octree t) {
  if (!handle_ok(t)) return;
  int dev = -1;
  (void)hipGetDevice(&dev);
  (void)hipSetDevice(t->device);
  (void)hipDeviceSynchronize();
  release(t);
  if (dev >= 0) (void)hipSetDevice(dev);
}

msp_status msp_octree_info(msp_octree t, int64_t* n_neurons, int64_t* n_nodes) {
  if (!handle_ok(t)) return MSP_ERR_INVALID;
  if (n_neurons) *n_neurons = t->n;
  if (n_nodes) *n_nodes = t->N;
  return MSP_OK;
}

msp_status msp_last_device_error(msp_octree t) {
  if (!handle_ok(t)) return MSP_ERR_INVALID;
  int32_t h = 0;
  MSP_HIP_TRY(hipMemcpy(&h, t->err, sizeof(int32_t), hipMemcpyDeviceToHost));
  return h ? MSP_ERR_DEVICE : MSP_OK;
}

msp_status msp_update_vacant_counts(msp_octree t, const int32_t* vac_dend_exc,
                                    const int32_t* vac_dend_inh, hipStream_t s) {
  if (!handle_ok(t) || !vac_dend_exc || !vac_dend_inh) return MSP_ERR_INVALID;
  for (int k = kMaxDepth; k >= 0; --k) {
    const int64_t cnt = t->level_off[k + 1] - t->level_off[k];
    if (cnt == 0) continue;
    refresh_level_k<<<grid_for(cnt, kRefreshBlock), kRefreshBlock, 0, s>>>(
        t->level_nodes + t->level_off[k], cnt, t->rec[0], t->rec[1], t->nbeg, t->nend, t->order,
        t->pos, vac_dend_exc, vac_dend_inh, t->vs[0], t->vs[1], t->err);
    MSP_HIP_TRY(hipGetLastError());
  }
  t->refreshed = true;
  return MSP_OK;
}

msp_status msp_find_targets_diag(msp_octree t, const uint8_t* neuron_type,
                                 const int32_t* vac_axon, double sigma_um, double theta,
                                 uint64_t seed, uint64_t step, int32_t* target_out,
                                 int64_t* elem_offset_out, int64_t capacity_S,
                                 const msp_search_diag* diag, hipStream_t s) {
  if (!handle_ok(t) || !neuron_type || !vac_axon || !elem_offset_out) return MSP_ERR_INVALID;
  if (!t->refreshed) return MSP_ERR_INVALID;
  if (!std::isfinite(sigma_um) || !(sigma_um > 0.0) || !std::isfinite(theta) || !(theta >= 0.0))
    return MSP_ERR_INVALID;
  if (capacity_S < 0) return MSP_ERR_INVALID;
  const int64_t n = t->n;
  Temp flag(s), p0(s), p1(s), work(s), ck(s);
  MSP_HIP_TRY(flag.alloc(sizeof(int32_t) * (4 + kXcd)));
  MSP_HIP_TRY(hipMemsetAsync(flag.p, 0, sizeof(int32_t) * (4 + kXcd), s));
  check_axon_k<<<grid_for(n, 256), 256, 0, s>>>(vac_axon, neuron_type, n, flag.as<int32_t>());
  MSP_HIP_TRY(hipGetLastError());
  MSP_HIP_TRY((exclusive_scan<int64_t, int32_t, CountPos>(vac_axon, elem_offset_out, n, CountPos(),
                                                          true, s)));
  int64_t S = 0;
  int32_t bad = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&S, elem_offset_out + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipMemcpyAsync(&bad, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  if (bad) return MSP_ERR_INVALID;
  if (S > capacity_S) return MSP_ERR_CAPACITY;
  if (S == 0) return MSP_OK;
  if (!target_out) return MSP_ERR_INVALID;

  MSP_HIP_TRY(p0.alloc(sizeof(int32_t) * (n + 1)));
  MSP_HIP_TRY(p1.alloc(sizeof(int32_t) * (n + 1)));
  const int64_t slots = n + 2 * kWave;
  MSP_HIP_TRY(work.alloc(sizeof(int32_t) * slots));
  MSP_HIP_TRY(hipMemsetAsync(work.p, 0xFF, sizeof(int32_t) * slots, s));
  MSP_HIP_TRY((exclusive_scan<int32_t, int32_t, SrcFlag>(t->order, p0.as<int32_t>(), n,
                                                         SrcFlag{vac_axon, neuron_type, 0}, true, s)));
  MSP_HIP_TRY((exclusive_scan<int32_t, int32_t, SrcFlag>(t->order, p1.as<int32_t>(), n,
                                                         SrcFlag{vac_axon, neuron_type, 1}, true, s)));
  int32_t* tiles = flag.as<int32_t>() + 1;
  int32_t* nslots = flag.as<int32_t>() + 2;
  int32_t* queue = flag.as<int32_t>() + 4;
  worklist_k<<<grid_for(n, 256), 256, 0, s>>>(t->order, vac_axon, neuron_type, n,
                                              p0.as<int32_t>(), p1.as<int32_t>(),
                                              work.as<int32_t>(), tiles);
  MSP_HIP_TRY(hipGetLastError());
  const bool simple = use_simple_kernel();

  SearchArgs A;
  A.rec[0] = t->rec[0];
  A.rec[1] = t->rec[1];
  A.vs[0] = t->vs[0];
  A.vs[1] = t->vs[1];
  A.pos = t->pos;
  A.order = t->order;
  A.nbeg = t->nbeg;
  A.nend = t->nend;
  A.leaf_of = t->leaf_of;
  A.type = neuron_type;
  A.vac_axon = vac_axon;
  A.elem_off = elem_offset_out;
  A.work = work.as<int32_t>();
  A.work_count = nslots;
  A.target = target_out;
  A.err = t->err;
  A.L2 = t->box_edge * t->box_edge;
  A.theta2 = theta * theta;
  A.k2 = kLog2e / (sigma_um * sigma_um);
  A.seed = seed;
  A.step = step;
  DiagOut D{};
  bool any = false;
  if (diag) {
    D = DiagOut{diag->z0, diag->levels, diag->visits, diag->opens, diag->visits0, diag->opens0};
    any = D.z0 || D.levels || D.visits || D.opens || D.visits0 || D.opens0;
  }
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  const bool timed = diag && diag->kernel_ms;
  if (timed)
    for (auto& e : ev) MSP_HIP_TRY(hipEventCreate(&e));
  // the coherent sweep needs the exact tile count to size its checkpoint buffers
  int32_t ntiles = 0;
  if (!simple) {
    MSP_HIP_TRY(hipMemcpyAsync(&ntiles, tiles, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MSP_HIP_TRY(hipStreamSynchronize(s));
  }
  SweepOut W{};
  unsigned sweep_blocks = 0;
  if (simple) {
    tiles_to_slots_k<<<1, 64, 0, s>>>(tiles, nslots);
  } else {
    int ncu = 0, per_cu = 0;
    MSP_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, t->device));
    MSP_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, any ? (const void*)search_sweep_k<true> : (const void*)search_sweep_k<false>,
        kWaveBlock, 0));
    if (per_cu < 1) per_cu = 1;
    int64_t blocks = (int64_t)ncu * per_cu;
    const int64_t need = ((int64_t)ntiles + (kWaveBlock / kWave) - 1) / (kWaveBlock / kWave);
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    sweep_blocks = (unsigned)blocks;
    const int64_t nt = ntiles > 0 ? ntiles : 1;
    const int64_t ns = nt * kWave;
    const int64_t nc = nt * kCkpt * kWave;
    const size_t bytes = sizeof(double) * (size_t)(ns + nc) +
                         sizeof(int32_t) * (size_t)(2 * ns + nt + nt * kCkpt + nc);
    MSP_HIP_TRY(ck.alloc(bytes));
    W.Z = ck.as<double>();
    W.ck_P = W.Z + ns;
    W.v0 = reinterpret_cast<int32_t*>(W.ck_P + nc);
    W.o0 = W.v0 + ns;
    W.nck = W.o0 + ns;
    W.ck_x = W.nck + nt;
    W.ck_me = W.ck_x + nt * kCkpt;
    W.tile_count = tiles;
    W.queue = queue;
    W.wave_steps = diag ? reinterpret_cast<unsigned long long*>(diag->wave_steps) : nullptr;
  }
  if (timed) MSP_HIP_TRY(hipEventRecord(ev[0], s));
  if (simple) {
    if (any)
      search_simple_k<true><<<grid_for(slots, 256), 256, 0, s>>>(A, D);
    else
      search_simple_k<false><<<grid_for(slots, 256), 256, 0, s>>>(A, D);
  } else if (ntiles > 0) {
    const unsigned draw_grid = grid_for((int64_t)ntiles * kWave, 256);
    if (any)
      search_sweep_k<true><<<sweep_blocks, kWaveBlock, 0, s>>>(A, W);
    else
      search_sweep_k<false><<<sweep_blocks, kWaveBlock, 0, s>>>(A, W);
    if (timed) MSP_HIP_TRY(hipEventRecord(ev[1], s));
    if (any)
      search_draw_k<true><<<draw_grid, 256, 0, s>>>(A, D, W);
    else
      search_draw_k<false><<<draw_grid, 256, 0, s>>>(A, D, W);
  }
  if (timed && (simple || ntiles == 0)) MSP_HIP_TRY(hipEventRecord(ev[1], s));
  hipError_t le = hipGetLastError();
  if (timed) {
    float a = 0.0f, b = 0.0f;
    (void)hipEventRecord(ev[2], s);
    (void)hipEventSynchronize(ev[2]);
    (void)hipEventElapsedTime(&a, ev[0], ev[1]);
    (void)hipEventElapsedTime(&b, ev[1], ev[2]);
    diag->kernel_ms[0] = a;
    diag->kernel_ms[1] = b;
    for (auto& e : ev) (void)hipEventDestroy(e);
  }
  MSP_HIP_TRY(le);
  return MSP_OK;
}

msp_status msp_find_targets(msp_octree t, const uint8_t* neuron_type, const int32_t* vac_axon,
                            double sigma_um, double theta, uint64_t seed, uint64_t step,
                            int32_t* target_out, int64_t* elem_offset_out, int64_t capacity_S,
                            hipStream_t s) {
  return msp_find_targets_diag(t, neuron_type, vac_axon, sigma_um, theta, seed, step, target_out,
                               elem_offset_out, capacity_S, nullptr, s);
}

msp_status msp_commit_synapses_ex(const int32_t* target, const int64_t* elem_offset,
                                  const uint8_t* neuron_type, int64_t n, int32_t* vac_axon,
                                  int32_t* vac_exc, int32_t* vac_inh, uint64_t seed,
                                  uint64_t step, int32_t* syn_src, int32_t* syn_tgt,
                                  uint8_t* syn_type, int64_t syn_capacity, int64_t* n_formed,
                                  uint8_t* accepted_out, hipStream_t s) {
  if (!elem_offset || !neuron_type || !vac_axon || !vac_exc || !vac_inh || !n_formed)
    return MSP_ERR_INVALID;
  if (n < 1 || n > MSP_MAX_NEURONS || syn_capacity < 0) return MSP_ERR_INVALID;
  int64_t S = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&S, elem_offset + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  if (S < 0) return MSP_ERR_INVALID;
  if (S == 0) {
    MSP_HIP_TRY(hipMemsetAsync(n_formed, 0, sizeof(int64_t), s));
    return MSP_OK;
  }
  if (!target) return MSP_ERR_INVALID;
  Temp src_of(s), key(s), prio(s), cnt(s), seg_off(s), seg(s), acc(s), dst(s), err(s);
  MSP_HIP_TRY(src_of.alloc(sizeof(int32_t) * S));
  MSP_HIP_TRY(key.alloc(sizeof(int64_t) * S));
  MSP_HIP_TRY(prio.alloc(sizeof(uint64_t) * S));
  MSP_HIP_TRY(cnt.alloc(sizeof(int32_t) * 2 * n));
  MSP_HIP_TRY(seg_off.alloc(sizeof(int32_t) * (2 * n + 1)));
  MSP_HIP_TRY(seg.alloc(sizeof(int32_t) * S));
  MSP_HIP_TRY(acc.alloc(sizeof(uint8_t) * S));
  MSP_HIP_TRY(dst.alloc(sizeof(int64_t) * (S + 1)));
  MSP_HIP_TRY(err.alloc(sizeof(int32_t)));
  MSP_HIP_TRY(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * 2 * n, s));
  MSP_HIP_TRY(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
  src_of_k<<<grid_for(n, kCommitBlock), kCommitBlock, 0, s>>>(elem_offset, n, src_of.as<int32_t>());
  req_key_k<<<grid_for(S, kCommitBlock), kCommitBlock, 0, s>>>(
      target, elem_offset, src_of.as<int32_t>(), neuron_type, S, n, seed, step, key.as<int64_t>(),
      prio.as<uint64_t>(), cnt.as<int32_t>(), err.as<int32_t>());
  MSP_HIP_TRY(hipGetLastError());
  MSP_HIP_TRY((exclusive_scan<int32_t, int32_t, Ident<int32_t>>(cnt.as<int32_t>(),
                                                                seg_off.as<int32_t>(), 2 * n,
                                                                Ident<int32_t>(), true, s)));
  // cursor = copy of the group offsets
  MSP_HIP_TRY(hipMemcpyAsync(cnt.p, seg_off.p, sizeof(int32_t) * 2 * n, hipMemcpyDeviceToDevice, s));
  req_scatter_k<<<grid_for(S, kCommitBlock), kCommitBlock, 0, s>>>(key.as<int64_t>(), S,
                                                                   cnt.as<int32_t>(),
                                                                   seg.as<int32_t>());
  req_rank_k<<<grid_for(S, kCommitBlock), kCommitBlock, 0, s>>>(
      key.as<int64_t>(), prio.as<uint64_t>(), seg_off.as<int32_t>(), seg.as<int32_t>(), S,
      vac_exc, vac_inh, acc.as<uint8_t>());
  MSP_HIP_TRY(hipGetLastError());
  MSP_HIP_TRY((exclusive_scan<int64_t, uint8_t, AccFlag>(acc.as<uint8_t>(), dst.as<int64_t>(), S,
                                                         AccFlag(), true, s)));
  int64_t formed = 0;
  int32_t bad = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&formed, dst.as<int64_t>() + S, sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipMemcpyAsync(&bad, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  if (bad) return MSP_ERR_INVALID;
  if (formed > syn_capacity) return MSP_ERR_CAPACITY;
  if (formed > 0 && (!syn_src || !syn_tgt || !syn_type)) return MSP_ERR_INVALID;
  commit_write_k<<<grid_for(S, kCommitBlock), kCommitBlock, 0, s>>>(
      acc.as<uint8_t>(), dst.as<int64_t>(), key.as<int64_t>(), src_of.as<int32_t>(), S, vac_axon,
      vac_exc, vac_inh, syn_src, syn_tgt, syn_type, accepted_out);
  copy_scalar_k<<<1, 64, 0, s>>>(dst.as<int64_t>() + S, n_formed);
  MSP_HIP_TRY(hipGetLastError());
  return MSP_OK;
}

msp_status msp_commit_synapses(const int32_t* target, const int64_t* elem_offset,
                               const uint8_t* neuron_type, int64_t n, int32_t* vac_axon,
                               int32_t* vac_exc, int32_t* vac_inh, uint64_t seed, uint64_t step,
                               int32_t* syn_src, int32_t* syn_tgt, uint8_t* syn_type,
                               int64_t syn_capacity, int64_t* n_formed, hipStream_t s) {
  return msp_commit_synapses_ex(target, elem_offset, neuron_type, n, vac_axon, vac_exc, vac_inh,
                                seed, step, syn_src, syn_tgt, syn_type, syn_capacity, n_formed,
                                nullptr, s);
}

// ---------------------------------------------------------------------------- export
}  // extern "C"

namespace {
__global__ void export_topo_k(const int32_t* __restrict__ skip, const uint8_t* __restrict__ depth,
                              const int32_t* __restrict__ nbeg, const int32_t* __restrict__ nend,
                              int64_t N, int32_t* d, int64_t* b, int64_t* e, int64_t* se) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  if (d) d[x] = depth[x];
  if (b) b[x] = nbeg[x];
  if (e) e[x] = nend[x];
  if (se) se[x] = skip[x];
}

__global__ void export_agg_k(const NodeRec* __restrict__ r, int64_t N, int64_t* v, double* c) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  const NodeRec q = r[x];
  if (v) v[x] = q.v;
  if (c) {
    c[3 * x + 0] = q.x;
    c[3 * x + 1] = q.y;
    c[3 * x + 2] = q.z;
  }
}
}  // namespace

extern "C" {

msp_status msp_octree_export_topology(msp_octree t, int32_t* order, uint64_t* keys,
                                      int32_t* depth, int64_t* node_begin, int64_t* node_end,
                                      int64_t* subtree_end, hipStream_t s) {
  if (!handle_ok(t)) return MSP_ERR_INVALID;
  if (order)
    MSP_HIP_TRY(hipMemcpyAsync(order, t->order, sizeof(int32_t) * t->n, hipMemcpyDeviceToDevice, s));
  if (keys)
    MSP_HIP_TRY(hipMemcpyAsync(keys, t->keys, sizeof(uint64_t) * t->n, hipMemcpyDeviceToDevice, s));
  export_topo_k<<<grid_for(t->N, 256), 256, 0, s>>>(t->skip, t->depth, t->nbeg, t->nend, t->N,
                                                    depth, node_begin, node_end, subtree_end);
  MSP_HIP_TRY(hipGetLastError());
  return MSP_OK;
}

msp_status msp_octree_export_aggregates(msp_octree t, int32_t type, int64_t* count,
                                        double* centroid, hipStream_t s) {
  if (!handle_ok(t) || (type != 0 && type != 1)) return MSP_ERR_INVALID;
  export_agg_k<<<grid_for(t->N, 256), 256, 0, s>>>(t->rec[type], t->N, count, centroid);
  MSP_HIP_TRY(hipGetLastError());
  return MSP_OK;
}

}  // extern "C"
