// libmsp: C ABI entry points (declared in include/msp.h). One translation unit.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <new>
#include <vector>

#include "common.hpp"
#include "scan.hpp"
#include "build.hpp"
#include "refresh.hpp"
#include "search.hpp"
#include "search_wave.hpp"
#include "batch.hpp"
#include "attraction.hpp"
#include "commit.hpp"
#include "plasticity.hpp"
#include "update.hpp"
#include "activity.hpp"

using namespace msp;

namespace {

void carve_neurons(msp_octree_s* t, char* base, size_t* bytes) {
  Carver c{base};
  const int64_t n = t->n;
  t->pos = c.take<double>(3 * n);
  t->keys = c.take<uint64_t>(n);
  t->order = c.take<int32_t>(n);
  t->leaf_of = c.take<int32_t>(n);
  t->leaf_at = c.take<int32_t>(n);
  t->vs[0] = c.take<int32_t>(n);
  t->vs[1] = c.take<int32_t>(n);
  t->err = c.take<int32_t>(1);
  *bytes = c.off;
}

void carve_nodes(msp_octree_s* t, char* base, size_t* bytes) {
  Carver c{base};
  const int64_t N = t->N;
  // + a sentinel record at index N, then room for the search sweep's requests ahead of
  // its position (never written, never read into registers)
  t->rec[0] = c.take<NodeRec>(N + 1 + kAheadRecords);
  t->rec[1] = c.take<NodeRec>(N + 1 + kAheadRecords);
  t->skip = c.take<int32_t>(N);
  t->nbeg = c.take<int32_t>(N);
  t->nend = c.take<int32_t>(N);
  t->level_nodes = c.take<int32_t>(N);
  t->depth = c.take<uint8_t>(N);
  *bytes = c.off;
}

// Return the octree's memory to the library pool, ordered on `fs` (null: the library's
// own stream, for callers that have waited for every use), and delete the struct. The
// handle must already be unregistered (or never have been registered).
void release(msp_octree_s* t, hipStream_t fs = nullptr, bool on_caller_stream = false) {
  if (!t) return;
  if (!on_caller_stream && lib_stream(t->device, &fs) != hipSuccess) fs = nullptr;
  if (t->slab_n) (void)hipFreeAsync(t->slab_n, fs);
  if (t->slab_N) (void)hipFreeAsync(t->slab_N, fs);
  delete t;
}

struct NonNeg {                 // a count, negative ones taken as 0 (they are reported)
  __device__ int64_t operator()(int32_t a, int64_t) const { return a > 0 ? (int64_t)a : 0; }
};

__global__ void negative_k(const int32_t* __restrict__ a, int64_t n, int32_t* err) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && a[k] < 0) atomicOr(err, 1);
}

// Whether the walks must test for the source's own cell: always, unless theta <= 1/2
// and every position of the tree lies inside its cube (then that test never fires).
// The walks without the test also decide acceptance by a bound on d2 (accept_bound),
// which asks for L^2 < kAcceptL2Max as well.
bool own_cell_needed(const msp_octree_s* t, double theta) {
  return !(t->inside && theta * theta <= 0.25 && t->box_edge * t->box_edge < kAcceptL2Max);
}

// Fill the device descriptor of one simulation.
SimDesc make_desc(const msp_octree_s* t, const uint8_t* neuron_type, const int32_t* vac_axon,
                  double sigma_um, double theta, uint64_t seed, uint64_t step, int32_t* target_out,
                  int64_t* elem_offset_out, int64_t capacity_S) {
  SimDesc d{};
  d.rec[0] = t->rec[0];
  d.rec[1] = t->rec[1];
  d.vs[0] = t->vs[0];
  d.vs[1] = t->vs[1];
  d.pos = t->pos;
  d.order = t->order;
  d.keys = t->keys;
  d.nbeg = t->nbeg;
  d.nend = t->nend;
  d.leaf_of = t->leaf_of;
  d.own = own_cell_needed(t, theta) ? 1 : 0;
  d.inside = t->inside ? 1 : 0;
  d.err = t->err;
  d.type = neuron_type;
  d.vac_axon = vac_axon;
  d.elem_off = elem_offset_out;
  d.target = target_out;
  d.capacity = target_out ? capacity_S : 0;
  d.n = t->n;
  d.L2 = t->box_edge * t->box_edge;
  d.theta2 = theta * theta;
  d.acc_d2 = accept_bound(d.L2, d.theta2);
  d.k2 = kLog2e / (sigma_um * sigma_um);
  d.seed = seed;
  d.step = step;
  return d;
}

// Branch level of the two-phase search when the caller names none: restarts from
// cells at this depth or deeper run in a second pass, in cell order.
constexpr int kDefaultBranchLevel = kNoDefer;

// Persistent sweep blocks: occupancy x CUs (times `frac` in [0, 1]), at most one
// wave per unit (a tile's part).
hipError_t sweep_blocks_for(int device, bool diag, int64_t max_units, double frac,
                            unsigned* blocks_out) {
  int ncu = 0, per_cu = 0;
  hipError_t e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu,
      diag ? (const void*)search_sweep_k<true, kCkptMax, true>
           : (const void*)search_sweep_k<false, kCkptMax, true>,
      kWaveBlock, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  int64_t blocks = (int64_t)((double)ncu * per_cu * frac);
  const int64_t need = (max_units + (kWaveBlock / kWave) - 1) / (kWaveBlock / kWave);
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  *blocks_out = (unsigned)blocks;
  return hipSuccess;
}

// Checkpoint slots per region: kCkptMax if one region per tile fits in an eighth of the
// device's memory, else kCkptMin. More slots mean shorter re-walks in the draw kernel;
// the targets do not depend on the choice. Regions: one per tile, and as many more as
// that eighth holds up to twice that (automatic parts) or the forced parts' units, so
// that most launches cut into parts give every part a region of its own.
hipError_t ck_slots_for(int device, int64_t total_n, int nsims, int force, int* slots_out,
                        int64_t* regions_out) {
  static size_t mem[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  if (mem[device] == 0) {
    hipDeviceProp_t p;
    hipError_t e = hipGetDeviceProperties(&p, device);
    if (e != hipSuccess) return e;
    mem[device] = p.totalGlobalMem;
  }
  const int64_t mt = max_tiles_for(total_n, nsims);
  const double budget = (double)(mem[device] / 8);
  const int slots = (double)mt * kCkptMax * (double)kCkptSlotBytes <= budget ? kCkptMax : kCkptMin;
  const int64_t want = force >= 0 ? (mt << force) : 2 * mt;
  const int64_t fit = (int64_t)(budget / ((double)slots * (double)kCkptSlotBytes));
  *slots_out = slots;
  *regions_out = std::max(mt, std::min(want, fit));
  return hipSuccess;
}

// The working memory of the search (worklist and checkpoints: gigabytes for millions
// of neurons), the commit and the plasticity step is kept per device between calls and
// grown when a larger call needs more: mapping it anew on every call would cost more
// than the search, and returning hundreds of megabytes to the stream-ordered pool after
// every commit made the next pool free on the host take about a millisecond. Calls on
// one device take turns (a mutex held for the whole call); a call's stream waits for
// the kernels of the previous user before they are overwritten.
struct Workspace {
  std::mutex m;
  void* p = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;      // recorded after the last user's kernels
};

Workspace& workspace(int device) {
  static Workspace w[64];
  return w[device];
}

class WorkspaceLease {
 public:
  explicit WorkspaceLease(int device) : w_(workspace(device)), lock_(w_.m) {}
  WorkspaceLease(const WorkspaceLease&) = delete;
  WorkspaceLease& operator=(const WorkspaceLease&) = delete;
  hipError_t acquire(size_t bytes, hipStream_t s, void** out) {
    hipError_t e = hipSuccess;
    if (!w_.done && (e = hipEventCreateWithFlags(&w_.done, hipEventDisableTiming)) != hipSuccess)
      return e;
    if (bytes > w_.bytes) {
      if (w_.p) {
        if ((e = hipEventSynchronize(w_.done)) != hipSuccess) return e;
        (void)hipFree(w_.p);
        w_.p = nullptr;
        w_.bytes = 0;
      }
      const size_t want = bytes + bytes / 8;          // some room for a larger next call
      if ((e = hipMalloc(&w_.p, want)) != hipSuccess) {
        (void)hipGetLastError();
        if ((e = hipMalloc(&w_.p, bytes)) != hipSuccess) return e;
        w_.bytes = bytes;
      } else {
        w_.bytes = want;
      }
    } else if ((e = hipStreamWaitEvent(s, w_.done, 0)) != hipSuccess) {
      return e;
    }
    s_ = s;
    leased_ = true;
    *out = w_.p;
    return hipSuccess;
  }
  ~WorkspaceLease() {
    if (leased_) (void)hipEventRecord(w_.done, s_);
  }

 private:
  Workspace& w_;
  std::lock_guard<std::mutex> lock_;
  hipStream_t s_ = nullptr;
  bool leased_ = false;
};

// Working memory of msp_find_targets_noalloc: one fixed array per device, part of the
// code object (no allocation call). Sized for a search over MSP_NOALLOC_MAX_NEURONS
// neurons with kCkptMin checkpoint slots per tile, plus its descriptor and bases.
constexpr size_t kNoAllocBytes = (size_t)40 << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

// Device address of `scratch` on `device` (the array's name is a host-side stand-in,
// not a device address): resolved once per device with that device current.
hipError_t noalloc_scratch(int device, void** out) {
  static std::mutex m;
  static void* addr[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(m);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

// The octree's per-type vacancy counts and centroids from the vacant dendritic
// elements: leaves first, then the inner nodes level by level, deepest first.
hipError_t enqueue_refresh(msp_octree_s* t, const int32_t* vac_exc, const int32_t* vac_inh,
                           hipStream_t s) {
  refresh_leaves_k<<<grid_for(t->n, kRefreshBlock), kRefreshBlock, 0, s>>>(
      t->n, t->rec[0], t->rec[1], t->leaf_at, t->nbeg, t->nend, t->order, t->pos, vac_exc,
      vac_inh, t->vs[0], t->vs[1], t->err);
  hipError_t e = hipGetLastError();
  for (int k = kMaxDepth; k >= 0 && e == hipSuccess; --k) {
    const int64_t cnt = t->level_off[k + 1] - t->level_off[k];
    if (cnt == 0) continue;
    refresh_level_k<<<grid_for(cnt, kRefreshBlock), kRefreshBlock, 0, s>>>(
        t->level_nodes + t->level_off[k], cnt, t->rec[0], t->rec[1], t->err);
    e = hipGetLastError();
  }
  return e;
}

// The search's descriptor and neuron bases written by a kernel (arguments by value):
// no host-to-device copy.
__global__ void put_desc_k(SimDesc h, SimDesc* d, int64_t* base, int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *d = h;
    base[0] = 0;
    base[1] = n;
  }
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
    case MSP_ERR_TOO_LARGE:
      return "problem larger than the fixed working memory of the allocation-free entry point";
    default: return "unknown status";
  }
}

msp_status msp_sync(hipStream_t s) {
  MSP_HIP_TRY(hipStreamSynchronize(s));
  return MSP_OK;
}

msp_status msp_release_workspace(int32_t device) {
  int ndev = 0;
  MSP_HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev || device >= 64) return MSP_ERR_INVALID;
  Workspace& w = workspace(device);
  std::lock_guard<std::mutex> g(w.m);
  if (!w.p) return MSP_OK;
  int cur = -1;
  MSP_HIP_TRY(hipGetDevice(&cur));
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess && w.done) e = hipEventSynchronize(w.done);
  if (e == hipSuccess) e = hipFree(w.p);
  if (e == hipSuccess) {
    w.p = nullptr;
    w.bytes = 0;
  }
  (void)hipSetDevice(cur);
  MSP_HIP_TRY(e);
  return MSP_OK;
}

msp_status msp_build_octree(const double* pos, int64_t n, const double box_min[3],
                            double box_edge, int32_t leaf_size, hipStream_t s, msp_octree* out) {
  if (!out) return MSP_ERR_INVALID;
  *out = nullptr;
  if (!pos || !box_min || n < 1 || n > MSP_MAX_NEURONS || leaf_size != 1) return MSP_ERR_INVALID;
  // the cube edge's square lowered by 4^21 (the finest cell's) must stay a normal double
  if (!std::isfinite(box_edge) || !(box_edge >= std::ldexp(1.0, -480)) ||
      !(box_edge <= std::ldexp(1.0, 480)))
    return MSP_ERR_INVALID;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(box_min[a])) return MSP_ERR_INVALID;

  msp_octree_s* t = new (std::nothrow) msp_octree_s();
  if (!t) return MSP_ERR_OOM;
  std::memset(t, 0, sizeof(*t));
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

  size_t bytes = 0;
  carve_neurons(t, nullptr, &bytes);
  TRY(pool_alloc(&t->slab_n, bytes, s));
  carve_neurons(t, static_cast<char*>(t->slab_n), &bytes);
  TRY(hipMemsetAsync(t->err, 0, sizeof(int32_t), s));
  {
    // every temporary of the build in one pool block (one allocation, one free)
    const size_t b_k1 = align_up(sizeof(uint64_t) * n), b_v1 = align_up(sizeof(int32_t) * n),
                 b_ws = align_up(radix_sort_ws_bytes(n)), b_cnt = align_up(sizeof(int32_t) * n),
                 b_base = align_up(sizeof(int32_t) * (n + 1)),
                 b_lvl = align_up(sizeof(int32_t) * 2 * (kMaxDepth + 1)),
                 b_out = align_up(sizeof(int32_t)), b_scan = align_up(scan_tmp_bytes<int32_t>(n));
    Temp tmp(s);
    TRY(tmp.alloc(b_k1 + b_v1 + b_ws + b_cnt + b_base + b_lvl + b_out + b_scan));
    char* tp = tmp.as<char>();
    uint64_t* k1 = reinterpret_cast<uint64_t*>(tp);
    int32_t* v1 = reinterpret_cast<int32_t*>(tp + b_k1);
    void* sort_ws = tp + b_k1 + b_v1;
    int32_t* cntp = reinterpret_cast<int32_t*>(tp + b_k1 + b_v1 + b_ws);
    int32_t* basep = reinterpret_cast<int32_t*>(tp + b_k1 + b_v1 + b_ws + b_cnt);
    int32_t* lcnt = reinterpret_cast<int32_t*>(tp + b_k1 + b_v1 + b_ws + b_cnt + b_base);
    int32_t* outside = reinterpret_cast<int32_t*>(tp + b_k1 + b_v1 + b_ws + b_cnt + b_base +
                                                  b_lvl);
    void* scan_ws = tp + b_k1 + b_v1 + b_ws + b_cnt + b_base + b_lvl + b_out;
    TRY(hipMemsetAsync(outside, 0, sizeof(int32_t), s));
    keys_k<<<grid_for(n, kBuildBlock), kBuildBlock, 0, s>>>(pos, n, box_min[0], box_min[1],
                                                            box_min[2], box_edge, t->pos, t->keys,
                                                            t->order, t->err, outside);
    TRY(hipGetLastError());
    TRY(radix_sort_pairs_ws(t->keys, t->order, k1, v1, n, 63, s, sort_ws));
    node_count_k<<<grid_for(n, kBuildBlock), kBuildBlock, 0, s>>>(t->keys, n, cntp);
    TRY(hipGetLastError());
    TRY((exclusive_scan<int32_t, int32_t, Ident<int32_t>>(cntp, basep, n, Ident<int32_t>(), true,
                                                          s, scan_ws)));
    int32_t N32 = 0, h_outside = 1;
    TRY(hipMemcpyAsync(&N32, basep + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TRY(hipMemcpyAsync(&h_outside, outside, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    double far = 0.0;
    for (int a = 0; a < 3; ++a)
      far = std::max(far, std::max(std::fabs(box_min[a]), std::fabs(box_min[a] + box_edge)));
    t->inside = h_outside == 0 && far <= std::ldexp(box_edge, 18);
    if (N32 < 1 || N32 >= kMaxNodes) {
      release(t);
      return MSP_ERR_INVALID;
    }
    const int64_t N = N32;
    t->N = N;
    carve_nodes(t, nullptr, &bytes);
    TRY(pool_alloc(&t->slab_N, bytes, s));
    carve_nodes(t, static_cast<char*>(t->slab_N), &bytes);
    TRY(hipMemsetAsync(t->rec[0] + N, 0, sizeof(NodeRec), s));
    TRY(hipMemsetAsync(t->rec[1] + N, 0, sizeof(NodeRec), s));
    TRY(hipMemsetAsync(lcnt, 0, sizeof(int32_t) * 2 * (kMaxDepth + 1), s));
    nodes_k<<<grid_for(n, kBuildBlock), kBuildBlock, 0, s>>>(t->keys, t->order, n,
                                                             basep, t->skip, t->depth,
                                                             t->nbeg, t->nend, t->leaf_of,
                                                             t->leaf_at);
    TRY(hipGetLastError());
    TRY(hipGetLastError());
    level_count_k<<<grid_for(N, kBuildBlock * kLevelItems), kBuildBlock, 0, s>>>(t->depth, t->skip,
                                                                                N, lcnt);
    TRY(hipGetLastError());
    int32_t hc[kMaxDepth + 1];
    TRY(hipMemcpyAsync(hc, lcnt, sizeof(hc), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    t->level_off[0] = 0;
    for (int k = 0; k <= kMaxDepth; ++k) t->level_off[k + 1] = t->level_off[k] + hc[k];
    if (t->level_off[kMaxDepth + 1] > N) {
      release(t);
      return MSP_ERR_HIP;
    }
    int32_t* cursor = lcnt + (kMaxDepth + 1);
    level_cursor_k<<<1, 1, 0, s>>>(lcnt, cursor);
    level_scatter_k<<<grid_for(N, kBuildBlock * kLevelItems), kBuildBlock, 0, s>>>(
        t->depth, t->skip, N, cursor, t->level_nodes);
    TRY(hipGetLastError());
    init_meta_k<<<grid_for(N, kBuildBlock), kBuildBlock, 0, s>>>(t->skip, t->depth, t->nbeg,
                                                                 t->nend, t->order, N, t->rec[0],
                                                                 t->rec[1]);
    TRY(hipGetLastError());
  }
#undef TRY
  handle_register(t, HandleKind::kOctree);
  *out = t;
  return MSP_OK;
}

void msp_free_octree(msp_octree t) {
  if (!handle_take(t, HandleKind::kOctree)) return;
  int dev = -1;
  (void)hipGetDevice(&dev);
  (void)hipSetDevice(t->device);
  (void)hipDeviceSynchronize();
  release(t);
  if (dev >= 0) (void)hipSetDevice(dev);
}

msp_status msp_free_octree_async(msp_octree t, hipStream_t s) {
  if (!handle_take(t, HandleKind::kOctree)) return MSP_ERR_INVALID;
  int dev = -1;
  (void)hipGetDevice(&dev);
  (void)hipSetDevice(t->device);
  release(t, s, true);
  if (dev >= 0) (void)hipSetDevice(dev);
  return MSP_OK;
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
  MSP_HIP_TRY(enqueue_refresh(t, vac_dend_exc, vac_dend_inh, s));
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

  // the plain search is the batch of one simulation
  SimDesc h = make_desc(t, neuron_type, vac_axon, sigma_um, theta, seed, step, target_out,
                        elem_offset_out, capacity_S);
  bool any = false;
  if (diag) {
    h.diag = DiagOut{diag->z0, diag->levels, diag->visits, diag->opens, diag->visits0,
                     diag->opens0, diag->entries0};
    any = h.diag.z0 || h.diag.levels || h.diag.visits || h.diag.opens || h.diag.visits0 ||
          h.diag.opens0 || h.diag.entries0;
  }
  const int64_t hbase[2] = {0, n};
  int force = -1;                       // parts per tile: automatic
  if (diag && diag->parts_per_tile != 0) {
    const int pp = diag->parts_per_tile;
    if (pp != 1 && pp != 2 && pp != 4 && pp != 8) return MSP_ERR_INVALID;
    force = pp == 1 ? 0 : pp == 2 ? 1 : pp == 4 ? 2 : 3;
  }
  int slots = 0;
  int64_t regions = 0;
  MSP_HIP_TRY(ck_slots_for(t->device, n, 1, force, &slots, &regions));
  WorkspaceLease ws(t->device);
  void* scratch = nullptr;
  // the workspace also holds the simulation descriptor and the neuron bases
  const size_t body = scratch_sizes(n, 1, slots, force, regions).total;
  MSP_HIP_TRY(ws.acquire(body + align_up(sizeof(SimDesc)) + align_up(sizeof(hbase)), s,
                         &scratch));
  SimDesc* dsim = reinterpret_cast<SimDesc*>(static_cast<char*>(scratch) + body);
  int64_t* dbase = reinterpret_cast<int64_t*>(static_cast<char*>(scratch) + body +
                                              align_up(sizeof(SimDesc)));
  MSP_HIP_TRY(hipMemcpyAsync(dsim, &h, sizeof(SimDesc), hipMemcpyHostToDevice, s));
  MSP_HIP_TRY(hipMemcpyAsync(dbase, hbase, sizeof(hbase), hipMemcpyHostToDevice, s));
  SearchScratch S = carve(scratch, n, 1, slots, dsim, dbase, force, regions);
  S.own_cell = own_cell_needed(t, theta);
  if (any) S.W.wave_steps = reinterpret_cast<unsigned long long*>(diag->wave_steps);
  MSP_HIP_TRY(enqueue_prep(S, n, s, force));
  int32_t status = 0, ntiles = 0, nunits = 0;
  int64_t total_S = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&status, S.B.status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipMemcpyAsync(&ntiles, S.counters, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipMemcpyAsync(&nunits, S.W.unit_count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipMemcpyAsync(&total_S, elem_offset_out + n, sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  if (status & kSimInvalid) return MSP_ERR_INVALID;
  if (status & kSimCapacity) return MSP_ERR_CAPACITY;
  if (diag && diag->phase2_requests)
    MSP_HIP_TRY(hipMemsetAsync(diag->phase2_requests, 0, sizeof(int64_t), s));

  const bool timed = diag && diag->kernel_ms;
  if (ntiles == 0) {
    if (timed) diag->kernel_ms[0] = diag->kernel_ms[1] = diag->kernel_ms[2] = 0.0f;
    return MSP_OK;
  }
  // two phases: restarts from cells at depth >= the branch level wait for a second
  // pass that takes them in cell order
  int depth = kDefaultBranchLevel;
  if (diag && diag->branch_level != 0) depth = diag->branch_level;
  const bool two = depth >= 1 && depth <= kMaxDepth && total_S < INT32_MAX;
  Temp req(s);
  constexpr int key_bits = 16;        // two radix passes; keys < 2^15 < none
  if (two) {
    int node_bits = 1;
    while ((1ll << node_bits) < t->N) ++node_bits;
    const size_t ks = align_up(sizeof(uint64_t) * total_S);
    const size_t vs = align_up(sizeof(int32_t) * total_S);
    const size_t ls = align_up(sizeof(uint8_t) * total_S);
    MSP_HIP_TRY(req.alloc(2 * ks + 5 * vs + ls + radix_sort_ws_bytes(total_S)));
    char* p = static_cast<char*>(req.p);
    DeferOut& D = S.W.defer;
    D.depth = depth;
    D.shift = std::max(0, node_bits - (key_bits - 1));
    D.none = (1ull << key_bits) - 1;
    D.key = reinterpret_cast<uint64_t*>(p);
    D.val = reinterpret_cast<int32_t*>(p + 2 * ks);
    D.src = reinterpret_cast<int32_t*>(p + 2 * ks + 2 * vs);
    D.elem = reinterpret_cast<int32_t*>(p + 2 * ks + 3 * vs);
    D.cell = reinterpret_cast<int32_t*>(p + 2 * ks + 4 * vs);
    D.level = reinterpret_cast<uint8_t*>(p + 2 * ks + 5 * vs);
  }
  unsigned blocks = 0;
  MSP_HIP_TRY(sweep_blocks_for(t->device, any, nunits, 1.0, &blocks));
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  if (timed) {
    for (auto& e : ev) MSP_HIP_TRY(hipEventCreate(&e));
    MSP_HIP_TRY(hipEventRecord(ev[0], s));
  }
  hipError_t le = enqueue_search(S, any, blocks, 256, s, timed ? ev[1] : nullptr);
  if (timed && le == hipSuccess) le = hipEventRecord(ev[2], s);
  if (two && le == hipSuccess) {
    const size_t ks = align_up(sizeof(uint64_t) * total_S);
    const size_t vs = align_up(sizeof(int32_t) * total_S);
    const DeferOut& D = S.W.defer;
    char* p = static_cast<char*>(req.p);
    le = radix_sort_pairs_ws(D.key, D.val, reinterpret_cast<uint64_t*>(p + ks),
                             reinterpret_cast<int32_t*>(p + 2 * ks + vs), total_S, key_bits, s,
                             p + 2 * ks + 5 * vs + align_up(sizeof(uint8_t) * total_S));
    if (le == hipSuccess) {
      if (any)
        search_phase2_k<true><<<grid_for(total_S, 256), 256, kRestartLds * 256, s>>>(S.B, S.W,
                                                                                   total_S);
      else
        search_phase2_k<false><<<grid_for(total_S, 256), 256, kRestartLds * 256, s>>>(S.B, S.W,
                                                                                    total_S);
      if (diag && diag->phase2_requests)
        phase2_count_k<<<1, 1, 0, s>>>(S.W, total_S, diag->phase2_requests);
      le = hipGetLastError();
    }
  }
  if (timed) {
    float a = 0.0f, b = 0.0f, c = 0.0f;
    (void)hipEventRecord(ev[3], s);
    (void)hipEventSynchronize(ev[3]);
    (void)hipEventElapsedTime(&a, ev[0], ev[1]);
    (void)hipEventElapsedTime(&b, ev[1], ev[2]);
    (void)hipEventElapsedTime(&c, ev[2], ev[3]);
    diag->kernel_ms[0] = a;
    diag->kernel_ms[1] = b;
    diag->kernel_ms[2] = c;
    for (auto& e : ev) (void)hipEventDestroy(e);
  }
  MSP_HIP_TRY(le);
  return MSP_OK;
}

msp_status msp_search_offsets(const int32_t* vac_axon, int64_t n, int64_t* elem_offset_out,
                              int64_t* S_out, hipStream_t s) {
  if (!vac_axon || !elem_offset_out || !S_out || n < 1 || n > MSP_MAX_NEURONS)
    return MSP_ERR_INVALID;
  Temp err(s);
  MSP_HIP_TRY(err.alloc(sizeof(int32_t)));
  fill_i32_k<<<1, 64, 0, s>>>(err.as<int32_t>(), 1, 0);
  negative_k<<<grid_for(n, 256), 256, 0, s>>>(vac_axon, n, err.as<int32_t>());
  MSP_HIP_TRY(hipGetLastError());
  MSP_HIP_TRY((exclusive_scan<int64_t, int32_t, NonNeg>(vac_axon, elem_offset_out, n, NonNeg(),
                                                       true, s)));
  int64_t S = 0;
  int32_t bad = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&S, elem_offset_out + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipMemcpyAsync(&bad, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  if (bad) return MSP_ERR_INVALID;
  *S_out = S;
  return MSP_OK;
}

msp_status msp_find_targets(msp_octree t, const uint8_t* neuron_type, const int32_t* vac_axon,
                            double sigma_um, double theta, uint64_t seed, uint64_t step,
                            int32_t* target_out, int64_t* elem_offset_out, int64_t capacity_S,
                            hipStream_t s) {
  return msp_find_targets_diag(t, neuron_type, vac_axon, sigma_um, theta, seed, step, target_out,
                               elem_offset_out, capacity_S, nullptr, s);
}

msp_status msp_find_targets_noalloc(msp_octree t, const uint8_t* neuron_type,
                                    const int32_t* vac_axon, double sigma_um, double theta,
                                    uint64_t seed, uint64_t step, int32_t* target_out,
                                    int64_t* elem_offset_out, int64_t capacity_S, hipStream_t s) {
  if (!handle_ok(t) || !neuron_type || !vac_axon || !elem_offset_out) return MSP_ERR_INVALID;
  if (!t->refreshed) return MSP_ERR_INVALID;
  if (!std::isfinite(sigma_um) || !(sigma_um > 0.0) || !std::isfinite(theta) || !(theta >= 0.0))
    return MSP_ERR_INVALID;
  if (capacity_S < 0) return MSP_ERR_INVALID;
  const int64_t n = t->n;
  if (n > MSP_NOALLOC_MAX_NEURONS) return MSP_ERR_TOO_LARGE;
  int cur = -1;
  MSP_HIP_TRY(hipGetDevice(&cur));
  if (cur != t->device) return MSP_ERR_INVALID;   // the array of the tree's device
  // the same layout as msp_find_targets' workspace, with kCkptMin slots and one
  // checkpoint region per tile; the descriptor and the neuron bases follow it
  const size_t body = scratch_sizes(n, 1, kCkptMin).total;
  const size_t need = body + align_up(sizeof(SimDesc)) + align_up(2 * sizeof(int64_t));
  if (need > kNoAllocBytes) return MSP_ERR_TOO_LARGE;
  void* base = nullptr;
  MSP_HIP_TRY(noalloc_scratch(t->device, &base));
  char* p = static_cast<char*>(base);
  SimDesc* dsim = reinterpret_cast<SimDesc*>(p + body);
  int64_t* dbase = reinterpret_cast<int64_t*>(p + body + align_up(sizeof(SimDesc)));
  const SimDesc h = make_desc(t, neuron_type, vac_axon, sigma_um, theta, seed, step, target_out,
                              elem_offset_out, capacity_S);
  put_desc_k<<<1, 64, 0, s>>>(h, dsim, dbase, n);
  MSP_HIP_TRY(hipGetLastError());
  SearchScratch S = carve(base, n, 1, kCkptMin, dsim, dbase);
  S.own_cell = own_cell_needed(t, theta);
  MSP_HIP_TRY(enqueue_prep(S, n, s));
  int32_t status = 0, ntiles = 0, nunits = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&status, S.B.status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipMemcpyAsync(&ntiles, S.counters, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipMemcpyAsync(&nunits, S.W.unit_count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  if (status & kSimInvalid) return MSP_ERR_INVALID;
  if (status & kSimCapacity) return MSP_ERR_CAPACITY;
  if (ntiles == 0) return MSP_OK;
  unsigned blocks = 0;
  MSP_HIP_TRY(sweep_blocks_for(t->device, false, nunits, 1.0, &blocks));
  MSP_HIP_TRY(enqueue_search(S, false, blocks, 256, s));
  return MSP_OK;
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
  // group offsets, cursors and request indices are int32
  if (S < 0 || S >= (int64_t)INT32_MAX) return MSP_ERR_INVALID;
  if (S == 0) {
    fill_i64_k<<<1, 64, 0, s>>>(n_formed, 1, 0);
    MSP_HIP_TRY(hipGetLastError());
    return MSP_OK;
  }
  if (!target) return MSP_ERR_INVALID;
  if (syn_capacity > 0 && (!syn_src || !syn_tgt || !syn_type)) return MSP_ERR_INVALID;
  // every temporary of the commit in the device's kept working memory
  size_t bytes = 0;
  (void)commit_ws(nullptr, n, S, &bytes);
  int dev = -1;
  MSP_HIP_TRY(hipGetDevice(&dev));
  WorkspaceLease lease(dev);
  void* wsp = nullptr;
  MSP_HIP_TRY(lease.acquire(bytes, s, &wsp));
  const CommitWs w = commit_ws(wsp, n, S, &bytes);
  MSP_HIP_TRY(enqueue_commit(w, target, elem_offset, neuron_type, n, host_count(S), vac_axon,
                             vac_exc, vac_inh, seed, host_step(step), syn_src, syn_tgt, syn_type,
                             syn_capacity, n_formed, accepted_out, s));
  int32_t flags = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&flags, w.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  if (flags & kErrArgs) return MSP_ERR_INVALID;
  if (flags & kCommitCapacity) return MSP_ERR_CAPACITY;
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

// ---------------------------------------------------------------------------- batched
struct msp_batch_s {
  int device;
  int32_t nsims;
  int32_t flags;
  int64_t total_n;
  std::vector<msp_sim> sims;
  SimDesc* h_sims;          // pinned staging of the descriptor table
  SimDesc* d_sims;
  int64_t* d_nbase;
  void* scratch;
  SearchScratch S;
  hipEvent_t staged;        // the descriptor upload of the last run has completed
  bool staged_pending;
  bool uploaded;            // the device table holds descriptors of the plan's sims
  unsigned sweep_blocks;
  int draw_block;
  int ck_slots;             // checkpoint slots per region
  int64_t ck_regions;       // checkpoint regions
  bool tuned;
  bool captured_own;        // own-cell test of the captured sweep
  hipGraphExec_t exec;
  bool captured;
  hipStream_t cap_stream;   // private stream for graph capture (the caller's may be the
                            // null stream, which cannot be captured)
};

namespace {

void batch_release(msp_batch_s* b) {
  if (!b) return;
  if (b->captured) (void)hipGraphExecDestroy(b->exec);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->staged) (void)hipEventDestroy(b->staged);
  if (b->h_sims) (void)hipHostFree(b->h_sims);
  if (b->d_sims) (void)hipFree(b->d_sims);
  if (b->d_nbase) (void)hipFree(b->d_nbase);
  if (b->scratch) (void)hipFree(b->scratch);
  delete b;
}

// A new theta and step in every descriptor of a batch (the rest is unchanged); the
// own-cell test as own_cell_needed decides it from the octree's `inside`.
__global__ void desc_theta_step_k(SimDesc* d, int n, double theta2, uint64_t step) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  d[k].theta2 = theta2;
  d[k].acc_d2 = accept_bound(d[k].L2, theta2);
  d[k].step = step;
  d[k].own = (d[k].inside && theta2 <= 0.25 && d[k].L2 < kAcceptL2Max) ? 0 : 1;
}

bool sim_ok(const msp_sim& m) {
  return handle_ok(m.tree) && m.tree->refreshed && m.neuron_type && m.vac_axon &&
         m.elem_offset_out && std::isfinite(m.sigma_um) && m.sigma_um > 0.0 && m.capacity_S >= 0;
}

hipError_t batch_enqueue(msp_batch_s* b, hipStream_t s) {
  hipError_t e = enqueue_prep(b->S, b->total_n, s);
  if (e != hipSuccess) return e;
  return enqueue_search(b->S, false, b->sweep_blocks, b->draw_block, s);
}

// Time launch shapes on the current descriptors and keep the fastest: the sweep's
// occupancy, the draw's block size and the checkpoint depth (slots per region: the
// plan's own, and kCkptMin where the plan holds more; the scratch carved for more
// slots holds fewer). Each shape is timed kTuneReps times after one untimed run, and
// its median counts. The targets do not depend on the shape.
constexpr int kTuneReps = 3;

hipError_t batch_autotune(msp_batch_s* b, hipStream_t s) {
  const double fracs[] = {1.0, 0.75, 0.5};
  const int draws[] = {256, 128, 64};
  const int slots_opts[] = {b->ck_slots, kCkptMin};
  const int n_slots = b->ck_slots == kCkptMin ? 1 : 2;
  const int64_t max_units = max_units_for(b->total_n, b->nsims);
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  float best = 1e30f;
  unsigned best_blocks = b->sweep_blocks;
  int best_draw = b->draw_block;
  int best_slots = b->S.W.ck_slots;
  for (int si = 0; si < n_slots && e == hipSuccess; ++si) {
    for (double f : fracs) {
      for (int d : draws) {
        unsigned blocks = 0;
        if ((e = sweep_blocks_for(b->device, false, max_units, f, &blocks)) != hipSuccess) break;
        b->sweep_blocks = blocks;
        b->draw_block = d;
        b->S.W.ck_slots = slots_opts[si];
        float t[kTuneReps + 1];
        for (int r = 0; r <= kTuneReps && e == hipSuccess; ++r) {
          if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
          if ((e = batch_enqueue(b, s)) != hipSuccess) break;
          if ((e = hipEventRecord(e1, s)) != hipSuccess) break;
          if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
          (void)hipEventElapsedTime(&t[r], e0, e1);
        }
        if (e != hipSuccess) break;
        std::sort(t + 1, t + kTuneReps + 1);       // run 0 is the untimed warm-up
        const float ms = t[1 + kTuneReps / 2];
        if (ms < best) {
          best = ms;
          best_blocks = blocks;
          best_draw = d;
          best_slots = slots_opts[si];
        }
      }
      if (e != hipSuccess) break;
    }
  }
  b->sweep_blocks = best_blocks;
  b->draw_block = best_draw;
  b->S.W.ck_slots = best_slots;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

}  // namespace

extern "C" {

msp_status msp_batch_create(const msp_sim* sims, int32_t n_sims, int32_t flags, msp_batch* out) {
  if (!out) return MSP_ERR_INVALID;
  *out = nullptr;
  if (!sims || n_sims < 1) return MSP_ERR_INVALID;
  for (int k = 0; k < n_sims; ++k)
    if (!sim_ok(sims[k])) return MSP_ERR_INVALID;
  int dev = -1;
  MSP_HIP_TRY(hipGetDevice(&dev));
  int64_t total = 0;
  std::vector<int64_t> base(n_sims + 1, 0);
  for (int k = 0; k < n_sims; ++k) {
    if (sims[k].tree->device != dev) return MSP_ERR_INVALID;
    base[k] = total;
    total += sims[k].tree->n;
  }
  base[n_sims] = total;
  if (total >= ((int64_t)1 << 31) - 4096) return MSP_ERR_INVALID;
  msp_batch_s* b = new (std::nothrow) msp_batch_s();
  if (!b) return MSP_ERR_OOM;
  b->device = dev;
  b->nsims = n_sims;
  b->flags = flags;
  b->total_n = total;
  b->sims.assign(sims, sims + n_sims);
  b->h_sims = nullptr;
  b->d_sims = nullptr;
  b->d_nbase = nullptr;
  b->scratch = nullptr;
  b->staged = nullptr;
  b->staged_pending = false;
  b->uploaded = false;
  b->tuned = false;
  b->captured = false;
  b->captured_own = true;
  b->cap_stream = nullptr;
  b->draw_block = 256;
  b->ck_slots = kCkptMin;
  hipError_t e = hipHostMalloc((void**)&b->h_sims, sizeof(SimDesc) * n_sims, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_sims, sizeof(SimDesc) * n_sims);
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_nbase, sizeof(int64_t) * (n_sims + 1));
  b->ck_regions = 0;
  if (e == hipSuccess) e = ck_slots_for(dev, total, n_sims, -1, &b->ck_slots, &b->ck_regions);
  if (e == hipSuccess)
    e = hipMalloc(&b->scratch, scratch_sizes(total, n_sims, b->ck_slots, -1, b->ck_regions).total);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
  b->cap_stream = nullptr;
  if (e == hipSuccess && (flags & MSP_BATCH_GRAPH))
    e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_nbase, base.data(), sizeof(int64_t) * (n_sims + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = sweep_blocks_for(dev, false, max_units_for(total, n_sims), 1.0, &b->sweep_blocks);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    batch_release(b);
    return e == hipErrorOutOfMemory ? MSP_ERR_OOM : MSP_ERR_HIP;
  }
  b->S = carve(b->scratch, total, n_sims, b->ck_slots, b->d_sims, b->d_nbase, -1, b->ck_regions);
  handle_register(b, HandleKind::kBatch);
  *out = b;
  return MSP_OK;
}

msp_status msp_find_targets_batched(msp_batch b, const msp_sim* sims, double theta,
                                    uint64_t step, hipStream_t s) {
  if (!handle_live(b, HandleKind::kBatch)) return MSP_ERR_INVALID;
  if (!std::isfinite(theta) || !(theta >= 0.0)) return MSP_ERR_INVALID;
  if (sims) {
    for (int k = 0; k < b->nsims; ++k)
      if (!sim_ok(sims[k]) || sims[k].tree != b->sims[k].tree) return MSP_ERR_INVALID;
    b->sims.assign(sims, sims + b->nsims);
  }
  bool own = false;
  for (int k = 0; k < b->nsims; ++k) own = own || own_cell_needed(b->sims[k].tree, theta);
  b->S.own_cell = own;
  if (b->captured && b->captured_own != own) {     // the captured sweep is the other variant
    MSP_HIP_TRY(hipStreamSynchronize(s));
    (void)hipGraphExecDestroy(b->exec);
    b->captured = false;
  }
  if (sims || !b->uploaded) {
    // new descriptors from the host; the staging buffer is reused: wait until the
    // previous upload has been read
    if (b->staged_pending) MSP_HIP_TRY(hipEventSynchronize(b->staged));
    for (int k = 0; k < b->nsims; ++k) {
      const msp_sim& m = b->sims[k];
      b->h_sims[k] = make_desc(m.tree, m.neuron_type, m.vac_axon, m.sigma_um, theta, m.seed,
                               step, m.target_out, m.elem_offset_out, m.capacity_S);
    }
    MSP_HIP_TRY(hipMemcpyAsync(b->d_sims, b->h_sims, sizeof(SimDesc) * b->nsims,
                               hipMemcpyHostToDevice, s));
    MSP_HIP_TRY(hipEventRecord(b->staged, s));
    b->staged_pending = true;
    b->uploaded = true;
  } else {
    // the same simulations: only theta and the step change, written on the device
    desc_theta_step_k<<<grid_for(b->nsims, 64), 64, 0, s>>>(b->d_sims, b->nsims, theta * theta,
                                                            step);
    MSP_HIP_TRY(hipGetLastError());
  }
  if ((b->flags & MSP_BATCH_AUTOTUNE) && !b->tuned) {
    MSP_HIP_TRY(batch_autotune(b, s));
    b->tuned = true;
  }
  if (b->flags & MSP_BATCH_GRAPH) {
    if (!b->captured) {
      hipGraph_t g;
      MSP_HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = batch_enqueue(b, b->cap_stream);
      hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        (void)hipGetLastError();
        return MSP_ERR_HIP;
      }
      e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return MSP_ERR_HIP;
      b->captured = true;
      b->captured_own = own;
    }
    MSP_HIP_TRY(hipGraphLaunch(b->exec, s));
    return MSP_OK;
  }
  MSP_HIP_TRY(batch_enqueue(b, s));
  return MSP_OK;
}

msp_status msp_batch_status(msp_batch b, hipStream_t s, int32_t* status_out) {
  if (!handle_live(b, HandleKind::kBatch)) return MSP_ERR_INVALID;
  std::vector<int32_t> st(b->nsims, 0);
  MSP_HIP_TRY(hipMemcpyAsync(st.data(), b->S.B.status, sizeof(int32_t) * b->nsims,
                             hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  msp_status first = MSP_OK;
  for (int k = 0; k < b->nsims; ++k) {
    const msp_status v = (st[k] & kSimInvalid) ? MSP_ERR_INVALID
                         : (st[k] & kSimCapacity) ? MSP_ERR_CAPACITY : MSP_OK;
    if (status_out) status_out[k] = v;
    if (first == MSP_OK) first = v;
  }
  return first;
}

void msp_batch_free(msp_batch b) {
  if (!handle_take(b, HandleKind::kBatch)) return;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  batch_release(b);
}

}  // extern "C"

// ---------------------------------------------------------------------------- attraction
namespace {

msp_status attraction(msp_octree t, const uint8_t* neuron_type, const int32_t* vac_axon,
                      double sigma_um, double theta, bool bwd, float* Z_out, const float* gZ,
                      float* dpos, double* dsigma, hipStream_t s) {
  if (!handle_ok(t) || !t->refreshed || !neuron_type || !vac_axon) return MSP_ERR_INVALID;
  if (!std::isfinite(sigma_um) || !(sigma_um > 0.0) || !std::isfinite(theta) || !(theta >= 0.0))
    return MSP_ERR_INVALID;
  if (bwd ? (!gZ || !dpos || !dsigma) : !Z_out) return MSP_ERR_INVALID;
  const int64_t n = t->n, N = t->N;
  Temp dsim(s), dbase(s), scratch(s), off(s), grads(s);
  MSP_HIP_TRY(off.alloc(sizeof(int64_t) * (n + 1)));
  // the search's preparation gives the worklist; targets are not written here
  SimDesc h = make_desc(t, neuron_type, vac_axon, sigma_um, theta, 0, 0,
                        reinterpret_cast<int32_t*>(off.p), off.as<int64_t>(), INT64_MAX);
  const int64_t hbase[2] = {0, n};
  MSP_HIP_TRY(dsim.alloc(sizeof(SimDesc)));
  MSP_HIP_TRY(dbase.alloc(sizeof(hbase)));
  // the worklist only: no draws, so no checkpoints
  MSP_HIP_TRY(scratch.alloc(scratch_sizes(n, 1, 0).total));
  MSP_HIP_TRY(hipMemcpyAsync(dsim.p, &h, sizeof(SimDesc), hipMemcpyHostToDevice, s));
  MSP_HIP_TRY(hipMemcpyAsync(dbase.p, hbase, sizeof(hbase), hipMemcpyHostToDevice, s));
  SearchScratch S = carve(scratch.p, n, 1, 0, dsim.as<SimDesc>(), dbase.as<int64_t>());
  MSP_HIP_TRY(enqueue_prep(S, n, s, -1, false));
  int32_t status = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&status, S.B.status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  if (status & kSimInvalid) return MSP_ERR_INVALID;

  if (!bwd) {
    // Z_i is the level-0 sum of the search: the sweep without checkpoints
    unsigned blocks = 0;
    MSP_HIP_TRY(sweep_blocks_for(t->device, false, max_units_for(n, 1), 1.0, &blocks));
    fill_i32_k<<<grid_for(n, 256), 256, 0, s>>>(reinterpret_cast<int32_t*>(Z_out), n, 0);
    S.own_cell = own_cell_needed(t, theta);
    launch_sweep<false, 0>(S, blocks, s);
    z_scatter_k<<<grid_for(S.B.max_slots, 256), 256, 0, s>>>(S.B, S.W, Z_out);
    MSP_HIP_TRY(hipGetLastError());
    return MSP_OK;
  }
  AttractArgs O{};
  O.gZ = gZ;
  O.two_over_s2 = 2.0 / (sigma_um * sigma_um);
  O.two_over_s3 = 2.0 / (sigma_um * sigma_um * sigma_um);
  O.N = N;
  O.unit_count = S.W.unit_count;
  const int64_t ng = 2 * N * 3, nh = 2 * N * 3, np = 3 * n;
  MSP_HIP_TRY(grads.alloc(sizeof(double) * (size_t)(kGradCopies * ng + nh + np)));
  O.G = grads.as<double>();
  double* H = O.G + kGradCopies * ng;
  O.dpos = H + nh;
  O.dsigma = dsigma;
  fill_f64_k<<<grid_for(kGradCopies * ng + nh + np, 256), 256, 0, s>>>(
      O.G, kGradCopies * ng + nh + np, 0.0);
  fill_f64_k<<<1, 64, 0, s>>>(dsigma, 1, 0.0);
  attract_bwd_k<<<grid_for(max_units_for(n, 1) * kWave, 256), 256, 0, s>>>(S.B, O);
  grad_sum_k<<<grid_for(ng, 256), 256, 0, s>>>(O.G, ng);
  for (int k = 0; k <= kMaxDepth; ++k) {
    const int64_t cnt = t->level_off[k + 1] - t->level_off[k];
    if (cnt == 0) continue;
    push_level_k<<<grid_for(cnt, 256), 256, 0, s>>>(t->level_nodes + t->level_off[k], cnt,
                                                     t->rec[0], t->rec[1], O.G, H, N);
  }
  push_leaves_k<<<grid_for(n, 256), 256, 0, s>>>(t->leaf_of, t->nbeg, t->nend, t->order,
                                                  t->vs[0], t->vs[1], H, N, n, O.dpos, dpos);
  MSP_HIP_TRY(hipGetLastError());
  return MSP_OK;
}

}  // namespace

extern "C" {

msp_status msp_attraction_fwd(msp_octree t, const uint8_t* neuron_type, const int32_t* vac_axon,
                              double sigma_um, double theta, float* Z_out, hipStream_t s) {
  return attraction(t, neuron_type, vac_axon, sigma_um, theta, false, Z_out, nullptr, nullptr,
                    nullptr, s);
}

msp_status msp_attraction_bwd(msp_octree t, const uint8_t* neuron_type, const int32_t* vac_axon,
                              double sigma_um, double theta, const float* gZ, float* dpos,
                              double* dsigma, hipStream_t s) {
  return attraction(t, neuron_type, vac_axon, sigma_um, theta, true, nullptr, gZ, dpos, dsigma,
                    s);
}

// ---------------------------------------------------------------------------
// Plasticity between updates
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
// The growth rule's constants from the parameters (the same double expressions as the
// definition, evaluated once).
PlastConst plast_const(const msp_plasticity_params& p) {
  PlastConst c;
  c.scale = (double)p.steps_per_update * p.growth_rate;
  c.xi = 0.5 * (p.growth_onset + p.target_calcium);
  c.zeta = (p.target_calcium - p.growth_onset) / (2.0 * std::sqrt(std::log(2.0)));
  c.ca_mean = p.calcium_mean;
  c.ca_sd = p.calcium_sd;
  c.delete_fraction = p.delete_fraction;
  return c;
}

// Parameters a plasticity step accepts.
bool plast_params_ok(const msp_plasticity_params& p) {
  const double vals[] = {p.growth_rate, p.target_calcium, p.growth_onset, p.calcium_mean,
                         p.calcium_sd, p.delete_fraction};
  for (double v : vals)
    if (!std::isfinite(v)) return false;
  return p.growth_onset < p.target_calcium && p.delete_fraction >= 0.0 &&
         p.delete_fraction <= 1.0 && p.steps_per_update >= 0;
}

ActParams act_params(const msp_activity_params& q) {
  ActParams P;
  P.a[0] = q.a_exc; P.b[0] = q.b_exc; P.c[0] = q.c_exc; P.d[0] = q.d_exc;
  P.a[1] = q.a_inh; P.b[1] = q.b_inh; P.c[1] = q.c_inh; P.d[1] = q.d_inh;
  P.w_e = q.w_exc;
  P.w_i = q.w_inh;
  P.mu = q.bg_mean;
  P.width = q.bg_width;
  P.beta = q.ca_beta;
  P.inv_tau = 1.0 / q.ca_tau;
  P.inv_delta = 1.0 / (double)q.epoch;
  P.delta = q.epoch;
  return P;
}
}  // namespace

extern "C" {

msp_status msp_plasticity_record(int64_t n, const int32_t* new_src, const int32_t* new_tgt,
                                 const uint8_t* new_type, int64_t m_new, int32_t* syn_src,
                                 int32_t* syn_tgt, uint8_t* syn_type, int64_t m, int64_t capacity,
                                 int32_t* bound, hipStream_t s) {
  if (n < 1 || m < 0 || m_new < 0 || !bound) return MSP_ERR_INVALID;
  if (m_new == 0) return MSP_OK;
  if (!new_src || !new_tgt || !new_type || !syn_src || !syn_tgt || !syn_type)
    return MSP_ERR_INVALID;
  if (m + m_new > capacity) return MSP_ERR_CAPACITY;
  MSP_HIP_TRY(hipMemcpyAsync(syn_src + m, new_src, sizeof(int32_t) * m_new,
                             hipMemcpyDeviceToDevice, s));
  MSP_HIP_TRY(hipMemcpyAsync(syn_tgt + m, new_tgt, sizeof(int32_t) * m_new,
                             hipMemcpyDeviceToDevice, s));
  MSP_HIP_TRY(hipMemcpyAsync(syn_type + m, new_type, sizeof(uint8_t) * m_new,
                             hipMemcpyDeviceToDevice, s));
  Temp err(s);
  MSP_HIP_TRY(err.alloc(sizeof(int32_t)));
  fill_i32_k<<<1, 64, 0, s>>>(err.as<int32_t>(), 1, 0);
  bind_k<<<grid_cap(m_new, kPlastBlock), kPlastBlock, 0, s>>>(new_src, new_tgt, new_type,
                                                            host_count(m_new), n, bound,
                                                            err.as<int32_t>());
  MSP_HIP_TRY(hipGetLastError());
  int32_t bad = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&bad, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  return bad ? MSP_ERR_INVALID : MSP_OK;
}

msp_status msp_plasticity_step(int64_t n, const msp_plasticity_params* params, uint64_t seed,
                               uint64_t step, double* z, int32_t* bound, int32_t* syn_src,
                               int32_t* syn_tgt, uint8_t* syn_type, int64_t m, int64_t* m_out,
                               int32_t* vac_axon, int32_t* vac_exc, int32_t* vac_inh,
                               hipStream_t s) {
  if (n < 1 || m < 0 || m >= ((int64_t)1 << 31) || !params || !z || !bound || !m_out ||
      !vac_axon || !vac_exc || !vac_inh)
    return MSP_ERR_INVALID;
  if (m > 0 && (!syn_src || !syn_tgt || !syn_type)) return MSP_ERR_INVALID;
  const msp_plasticity_params& p = *params;
  if (!plast_params_ok(p)) return MSP_ERR_INVALID;
  const PlastConst c = plast_const(p);
  int64_t* m_dev = nullptr;
  size_t bytes = 0;
  (void)plast_ws(nullptr, n, m, &bytes);
  int dev = -1;
  MSP_HIP_TRY(hipGetDevice(&dev));
  WorkspaceLease lease(dev);                  // the device's kept working memory
  void* wsp = nullptr;
  MSP_HIP_TRY(lease.acquire(bytes + align_up(sizeof(int64_t)), s, &wsp));
  const PlastWs w = plast_ws(wsp, n, m, &bytes);
  m_dev = reinterpret_cast<int64_t*>(static_cast<char*>(wsp) + bytes);
  MSP_HIP_TRY(enqueue_plasticity(w, n, c, seed, host_step(step), z, bound,
                                 SynList{syn_src, syn_tgt, syn_type}, host_count(m), m_dev,
                                 vac_axon, vac_exc, vac_inh, s));
  int64_t M = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&M, m_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  *m_out = M;
  return MSP_OK;
}


}  // extern "C"

// ---------------------------------------------------------------------------- update cycle
struct msp_cycle_s {
  int device;
  int32_t flags;
  msp_octree_s* t;
  int64_t n;
  const uint8_t* type;
  uint64_t seed;
  PlastConst pc;
  int64_t cap_S, cap_syn;
  msp_cycle_state st;
  void* mem;                // one allocation: everything below
  SimDesc* d_sim;
  int64_t* d_nbase;
  SearchScratch S;
  unsigned sweep_blocks;
  int64_t* elem_off;        // [n + 1]
  int32_t* target;          // [cap_S]
  CommitWs cw;
  SynList fresh;            // [cap_S] the update's new synapses
  int64_t* cnt;             // [2] searches, formed
  int32_t* rec_flags;       // [1]
  PlastWs pw;
  hipGraphExec_t exec;
  bool captured;
  hipStream_t cap_stream;   // private stream for graph capture
};

namespace {

// Start of an update: the step into the search descriptor, the record flags cleared.
__global__ void cycle_begin_k(SimDesc* d, const uint64_t* step, int32_t* rec_flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  d->step = *step;
  *rec_flags = 0;
}

// The searches the commit takes: none if the search reported an error (it then wrote
// no targets).
__global__ void cycle_searches_k(const int32_t* status, const int64_t* elem_off, int64_t n,
                                 int64_t* searches) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  *searches = *status ? 0 : elem_off[n];
}

// End of an update: its status bits into the caller's word, the counts out, the step on.
__global__ void cycle_end_k(const int32_t* search_status, const int32_t* commit_flags,
                            const int32_t* rec_flags, const int32_t* tree_err,
                            const int64_t* cnt, msp_cycle_state st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t b = 0;
  const int32_t ss = *search_status;
  if (ss & kSimInvalid) b |= MSP_CYCLE_SEARCH_INVALID;
  if (ss & kSimCapacity) b |= MSP_CYCLE_SEARCH_CAPACITY;
  if (*rec_flags & kRecordCapacity) b |= MSP_CYCLE_SYN_CAPACITY;
  if (*tree_err || (*commit_flags & kErrArgs)) b |= MSP_CYCLE_DEVICE;
  if (b) *st.status |= b;
  if (st.searches) *st.searches = cnt[0];
  if (st.formed) *st.formed = cnt[1];
  *st.step += 1;
}

void cycle_release(msp_cycle_s* c) {
  if (!c) return;
  if (c->captured) (void)hipGraphExecDestroy(c->exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->mem) (void)hipFree(c->mem);
  delete c;
}

// Carves the plan's memory (base null: sizes it).
size_t cycle_carve(msp_cycle_s* c, char* base, int slots, int64_t regions) {
  Carver cv{base};
  const int64_t n = c->n;
  void* search = cv.take_bytes(scratch_sizes(n, 1, slots, -1, regions).total);
  c->d_sim = cv.take<SimDesc>(1);
  c->d_nbase = cv.take<int64_t>(2);
  c->elem_off = cv.take<int64_t>(n + 1);
  c->target = cv.take<int32_t>(c->cap_S);
  size_t bytes = 0;
  (void)commit_ws(nullptr, n, c->cap_S, &bytes);
  void* cw = cv.take_bytes(bytes);
  c->fresh.src = cv.take<int32_t>(c->cap_S);
  c->fresh.tgt = cv.take<int32_t>(c->cap_S);
  c->fresh.type = cv.take<uint8_t>(c->cap_S);
  c->cnt = cv.take<int64_t>(2);
  c->rec_flags = cv.take<int32_t>(1);
  (void)plast_ws(nullptr, n, c->cap_syn, &bytes);
  void* pw = cv.take_bytes(bytes);
  if (base) {
    c->S = carve(search, n, 1, slots, c->d_sim, c->d_nbase, -1, regions);
    c->cw = commit_ws(cw, n, c->cap_S, &bytes);
    c->pw = plast_ws(pw, n, c->cap_syn, &bytes);
  }
  return cv.off;
}

// One update, kernels only (see msp_cycle_run).
hipError_t cycle_enqueue(msp_cycle_s* c, hipStream_t s) {
  const msp_cycle_state& st = c->st;
  const DevStep step{0, st.step};
  const int64_t n = c->n;
  cycle_begin_k<<<1, 64, 0, s>>>(c->d_sim, st.step, c->rec_flags);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = enqueue_refresh(c->t, st.vac_exc, st.vac_inh, s);
  if (e == hipSuccess) e = enqueue_prep(c->S, n, s);
  if (e == hipSuccess) e = enqueue_search(c->S, false, c->sweep_blocks, 256, s);
  if (e != hipSuccess) return e;
  cycle_searches_k<<<1, 64, 0, s>>>(c->S.B.status, c->elem_off, n, c->cnt);
  e = enqueue_commit(c->cw, c->target, c->elem_off, c->type, n, DevCount{c->cap_S, c->cnt},
                     st.vac_axon, st.vac_exc, st.vac_inh, c->seed, step, c->fresh.src,
                     c->fresh.tgt, c->fresh.type, c->cap_S, c->cnt + 1, nullptr, s);
  if (e != hipSuccess) return e;
  const SynList L{st.syn_src, st.syn_tgt, st.syn_type};
  const DevCount formed{c->cap_S, c->cnt + 1};
  record_k<<<grid_cap(c->cap_S, kPlastBlock), kPlastBlock, 0, s>>>(
      c->fresh, formed, L, st.m, c->cap_syn, n, st.bound, c->rec_flags);
  record_end_k<<<1, 64, 0, s>>>(formed, st.m, c->cap_syn);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = enqueue_plasticity(c->pw, n, c->pc, c->seed, step, st.z, st.bound, L,
                         DevCount{c->cap_syn, st.m}, st.m, st.vac_axon, st.vac_exc, st.vac_inh, s);
  if (e != hipSuccess) return e;
  cycle_end_k<<<1, 64, 0, s>>>(c->S.B.status, c->cw.flags, c->rec_flags, c->t->err, c->cnt, st);
  return hipGetLastError();
}

}  // namespace

extern "C" {

msp_status msp_cycle_create(msp_octree t, const uint8_t* neuron_type, double sigma_um,
                            double theta, uint64_t seed, const msp_plasticity_params* params,
                            int64_t search_capacity, int64_t syn_capacity,
                            const msp_cycle_state* state, int32_t flags, msp_cycle* out) {
  if (!out) return MSP_ERR_INVALID;
  *out = nullptr;
  if (!handle_ok(t) || !neuron_type || !params || !state) return MSP_ERR_INVALID;
  const msp_cycle_state& st = *state;
  if (!st.z || !st.bound || !st.syn_src || !st.syn_tgt || !st.syn_type || !st.m ||
      !st.vac_axon || !st.vac_exc || !st.vac_inh || !st.step || !st.status)
    return MSP_ERR_INVALID;
  if (!std::isfinite(sigma_um) || !(sigma_um > 0.0) || !std::isfinite(theta) || !(theta >= 0.0))
    return MSP_ERR_INVALID;
  if (!plast_params_ok(*params)) return MSP_ERR_INVALID;
  if (search_capacity < 1 || search_capacity >= (int64_t)INT32_MAX || syn_capacity < 1 ||
      syn_capacity >= ((int64_t)1 << 31))
    return MSP_ERR_INVALID;
  if ((flags & ~MSP_CYCLE_GRAPH) != 0) return MSP_ERR_INVALID;
  int dev = -1;
  MSP_HIP_TRY(hipGetDevice(&dev));
  if (dev != t->device) return MSP_ERR_INVALID;
  msp_cycle_s* c = new (std::nothrow) msp_cycle_s();
  if (!c) return MSP_ERR_OOM;
  c->device = dev;
  c->flags = flags;
  c->t = t;
  c->n = t->n;
  c->type = neuron_type;
  c->seed = seed;
  c->pc = plast_const(*params);
  c->cap_S = search_capacity;
  c->cap_syn = syn_capacity;
  c->st = st;
  c->mem = nullptr;
  c->captured = false;
  c->cap_stream = nullptr;
  int slots = 0;
  int64_t regions = 0;
  hipError_t e = ck_slots_for(dev, c->n, 1, -1, &slots, &regions);
  if (e == hipSuccess) e = hipMalloc(&c->mem, cycle_carve(c, nullptr, slots, regions));
  if (e == hipSuccess) {
    (void)cycle_carve(c, static_cast<char*>(c->mem), slots, regions);
    e = sweep_blocks_for(dev, false, max_units_for(c->n, 1), 1.0, &c->sweep_blocks);
  }
  if (e == hipSuccess && (flags & MSP_CYCLE_GRAPH))
    e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) {
    const SimDesc h = make_desc(t, neuron_type, st.vac_axon, sigma_um, theta, seed, 0, c->target,
                                c->elem_off, c->cap_S);
    const int64_t hbase[2] = {0, c->n};
    e = hipMemcpy(c->d_sim, &h, sizeof(SimDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(c->d_nbase, hbase, sizeof(hbase), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    cycle_release(c);
    return e == hipErrorOutOfMemory ? MSP_ERR_OOM : MSP_ERR_HIP;
  }
  c->S.own_cell = own_cell_needed(t, theta);
  handle_register(c, HandleKind::kCycle);
  *out = c;
  return MSP_OK;
}

msp_status msp_cycle_run(msp_cycle c, int32_t updates, hipStream_t s) {
  if (!handle_live(c, HandleKind::kCycle) || updates < 0) return MSP_ERR_INVALID;
  if (!handle_ok(c->t)) return MSP_ERR_INVALID;
  if (updates == 0) return MSP_OK;
  if (c->flags & MSP_CYCLE_GRAPH) {
    if (!c->captured) {
      hipGraph_t g;
      MSP_HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = cycle_enqueue(c, c->cap_stream);
      hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        (void)hipGetLastError();
        return MSP_ERR_HIP;
      }
      e = hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return MSP_ERR_HIP;
      c->captured = true;
    }
    for (int32_t k = 0; k < updates; ++k) MSP_HIP_TRY(hipGraphLaunch(c->exec, s));
    return MSP_OK;
  }
  for (int32_t k = 0; k < updates; ++k) MSP_HIP_TRY(cycle_enqueue(c, s));
  return MSP_OK;
}

void msp_cycle_free(msp_cycle c) {
  if (!handle_take(c, HandleKind::kCycle)) return;
  int dev = -1;
  (void)hipGetDevice(&dev);
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  cycle_release(c);
  if (dev >= 0) (void)hipSetDevice(dev);
}

msp_status msp_activity_init(int64_t n, const uint8_t* neuron_type,
                             const msp_activity_params* params, double* v, double* u,
                             double* calcium, uint8_t* spiked, int32_t* epoch_count, double* freq,
                             hipStream_t s) {
  if (n < 1 || !params || !neuron_type || !v || !u || !calcium || !spiked || !epoch_count ||
      !freq)
    return MSP_ERR_INVALID;
  Temp err(s);
  MSP_HIP_TRY(err.alloc(sizeof(int32_t)));
  fill_i32_k<<<1, 64, 0, s>>>(err.as<int32_t>(), 1, 0);
  act_init_k<<<grid_for(n, kActBlock), kActBlock, 0, s>>>(n, neuron_type, act_params(*params), v,
                                                          u, calcium, spiked, epoch_count, freq,
                                                          err.as<int32_t>());
  MSP_HIP_TRY(hipGetLastError());
  int32_t bad = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&bad, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  return bad ? MSP_ERR_INVALID : MSP_OK;
}

msp_status msp_activity_run(int64_t n, const uint8_t* neuron_type, const int32_t* rank,
                            int64_t m, const int32_t* syn_src, const int32_t* syn_tgt,
                            const uint8_t* syn_type, int32_t approx,
                            const msp_activity_params* params, uint64_t seed, uint64_t t0,
                            int32_t steps, double* v, double* u, double* calcium,
                            uint8_t* spiked, int32_t* epoch_count, double* freq,
                            int32_t* last_input, int64_t* spikes, hipStream_t s) {
  if (n < 1 || m < 0 || steps < 0 || approx < 0 || approx > 2 || !params || !neuron_type ||
      !v || !u || !calcium || !spiked || !epoch_count || !freq)
    return MSP_ERR_INVALID;
  if (m > 0 && (!syn_src || !syn_tgt || !syn_type)) return MSP_ERR_INVALID;
  if (approx == 1 && !rank) return MSP_ERR_INVALID;
  const msp_activity_params& q = *params;
  if (q.epoch < 1 || !(q.ca_tau > 0.0)) return MSP_ERR_INVALID;
  if (steps == 0) return MSP_OK;
  const ActParams P = act_params(q);
  Temp arr(s), err(s), part(s), grp(s);
  const int64_t nblocks = (int64_t)grid_for(n, kActBlock);
  // arrival counts (e, h) of two consecutive steps: step k consumes buffer k % 2 and its
  // spikes are delivered into the other
  MSP_HIP_TRY(arr.alloc(sizeof(int32_t) * 4 * n));
  MSP_HIP_TRY(err.alloc(sizeof(int32_t)));
  int32_t* buf = arr.as<int32_t>();
  MSP_HIP_TRY(hipMemsetAsync(buf, 0, sizeof(int32_t) * 4 * n, s));
  MSP_HIP_TRY(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
  if (spikes) {
    MSP_HIP_TRY(part.alloc(sizeof(int64_t) * nblocks));
    MSP_HIP_TRY(hipMemsetAsync(part.p, 0, sizeof(int64_t) * nblocks, s));
  }
  const int32_t* soff = nullptr;       // exact synapses by source (null: none)
  const int32_t* perm = nullptr;
  // approximated synapses: approx 1 packs them (index, endpoints, type); approx 2 reads
  // the caller's arrays
  const int32_t *a_idx = nullptr, *a_src = syn_src, *a_tgt = syn_tgt, *a_n = nullptr;
  const uint8_t* a_type = syn_type;
  if (m > 0) {
    const bool pack = approx == 1;
    const size_t z_off = align_up(sizeof(int32_t) * (n + 1)), z_cur = align_up(sizeof(int32_t) * n),
                 z_perm = align_up(sizeof(int32_t) * m),
                 z_rem = pack ? align_up(sizeof(uint8_t) * m) : 0,
                 z_pos = pack ? align_up(sizeof(int32_t) * (m + 1)) : 0,
                 z_pk = pack ? 3 * align_up(sizeof(int32_t) * m) + align_up(m) : 0,
                 z_scan = align_up(std::max(scan_tmp_bytes<int32_t>(n), scan_tmp_bytes<int32_t>(m)));
    MSP_HIP_TRY(grp.alloc(z_off + z_cur + z_perm + z_rem + z_pos + z_pk + z_scan));
    char* q = grp.as<char>();
    auto take = [&](size_t bytes) {
      char* r = q;
      q += bytes;
      return r;
    };
    int32_t* off = reinterpret_cast<int32_t*>(take(z_off));
    int32_t* cur = reinterpret_cast<int32_t*>(take(z_cur));
    int32_t* pm = reinterpret_cast<int32_t*>(take(z_perm));
    uint8_t* rem = pack ? reinterpret_cast<uint8_t*>(take(z_rem)) : nullptr;
    int32_t* rpos = pack ? reinterpret_cast<int32_t*>(take(z_pos)) : nullptr;
    char* pk = take(z_pk);
    void* scan_ws = take(z_scan);
    MSP_HIP_TRY(hipMemsetAsync(off, 0, sizeof(int32_t) * (n + 1), s));
    MSP_HIP_TRY(hipMemsetAsync(cur, 0, sizeof(int32_t) * n, s));
    act_setup_k<<<grid_for(m, kActBlock), kActBlock, 0, s>>>(n, m, syn_src, syn_tgt, syn_type,
                                                             rank, approx, off, rem,
                                                             err.as<int32_t>());
    MSP_HIP_TRY(hipGetLastError());
    if (pack) {
      const size_t zi = align_up(sizeof(int32_t) * m);
      int32_t* ai = reinterpret_cast<int32_t*>(pk);
      int32_t* as = reinterpret_cast<int32_t*>(pk + zi);
      int32_t* at = reinterpret_cast<int32_t*>(pk + 2 * zi);
      uint8_t* ay = reinterpret_cast<uint8_t*>(pk + 3 * zi);
      MSP_HIP_TRY((exclusive_scan<int32_t, uint8_t, Ident<int32_t>>(rem, rpos, m, Ident<int32_t>(),
                                                                    true, s, scan_ws)));
      act_pack_k<<<grid_for(m, kActBlock), kActBlock, 0, s>>>(m, syn_src, syn_tgt, syn_type, rem,
                                                              rpos, ai, as, at, ay);
      MSP_HIP_TRY(hipGetLastError());
      a_idx = ai;
      a_src = as;
      a_tgt = at;
      a_type = ay;
      a_n = rpos + m;
    }
    if (approx != 2) {
      MSP_HIP_TRY((exclusive_scan<int32_t, int32_t, Ident<int32_t>>(off, off, n, Ident<int32_t>(),
                                                                    true, s, scan_ws)));
      act_group_k<<<grid_for(m, kActBlock), kActBlock, 0, s>>>(n, m, syn_src, syn_tgt, syn_type,
                                                               rank, approx, off, cur, pm);
      act_deliver_k<<<grid_for(n, kActBlock), kActBlock, 0, s>>>(n, spiked, off, pm, syn_tgt,
                                                                 syn_type, buf, buf + n);
      MSP_HIP_TRY(hipGetLastError());
      soff = off;
      perm = pm;
    }
  }
  for (int32_t k = 0; k < steps; ++k) {
    const uint64_t t = t0 + (uint64_t)k;
    int32_t* e = buf + (int64_t)(k & 1) * 2 * n;
    int32_t* e2 = buf + (int64_t)((k + 1) & 1) * 2 * n;
    if (m > 0 && approx >= 1)
      act_approx_k<<<grid_for(m, kActBlock), kActBlock, 0, s>>>(
          n, m, a_src, a_tgt, a_type, a_idx, a_n, seed, t, freq, e, e + n);
    act_neuron_k<<<grid_for(n, kActBlock), kActBlock, 0, s>>>(
        n, neuron_type, P, seed, t, v, u, calcium, spiked, epoch_count, freq, e, e + n,
        k == steps - 1 ? last_input : nullptr, spikes ? part.as<int64_t>() : nullptr, soff, perm,
        syn_tgt, syn_type, e2, e2 + n);
    MSP_HIP_TRY(hipGetLastError());
  }
  if (spikes) {
    act_spikes_k<<<1, kActBlock, 0, s>>>(part.as<int64_t>(), nblocks, spikes);
    MSP_HIP_TRY(hipGetLastError());
  }
  int32_t bad = 0;
  MSP_HIP_TRY(hipMemcpyAsync(&bad, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  MSP_HIP_TRY(hipStreamSynchronize(s));
  return bad ? MSP_ERR_INVALID : MSP_OK;
}

}  // extern "C"
