// Shared device/host definitions of libmsp (one translation unit: msp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "msp.h"

namespace msp {

constexpr int kMaxDepth = 21;              // 21 bits per axis, 63-bit Morton keys
constexpr int kWave = 64;

// Per-node, per-type search record (32 bytes, one scalar load of 8 dwords).
//   x, y, z : float64 centroid of the type's vacant dendritic elements (leaf: the
//             neuron's position);
//   v       : vacant elements of the type below the node;
//   meta    : inner node -> bits 0..25 pre-order subtree end ("skip"), 26..30 depth;
//             leaf        -> bit 31 set; single neuron: bits 0..29 neuron id;
//                            bucket (coincident neurons) : bit 30 set, bits 0..29 node index.
struct alignas(32) NodeRec {
  double x, y, z;
  int32_t v;
  uint32_t meta;
};
static_assert(sizeof(NodeRec) == 32, "NodeRec must be 32 bytes");

constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kBucketBit = 0x40000000u;
constexpr uint32_t kIdMask = 0x3FFFFFFFu;
constexpr uint32_t kSkipBits = 26;
constexpr uint32_t kSkipMask = (1u << kSkipBits) - 1u;
constexpr int64_t kMaxNodes = (int64_t)1 << kSkipBits;

// device error flags (sticky, per octree)
constexpr int32_t kErrNonFinite = 1;
constexpr int32_t kErrNegative = 2;
constexpr int32_t kErrOverflow = 4;
constexpr int32_t kErrArgs = 8;

}  // namespace msp

struct msp_octree_s {
  int device;
  int64_t n;             // neurons
  int64_t N;             // nodes
  double box_min[3];
  double box_edge;
  // neuron arrays (device)
  double* pos;           // [n][3] by id
  uint64_t* keys;        // [n] sorted Morton keys
  int32_t* order;        // [n] ids in (key, id) order
  int32_t* leaf_of;      // [n] by id: leaf node holding the neuron
  int32_t* leaf_at;      // [n] by sorted position: leaf node holding it
  // topology (device), nodes in depth-first pre-order
  int32_t* skip;         // [N] subtree end
  uint8_t* depth;        // [N]
  int32_t* nbeg;         // [N] range in `order`
  int32_t* nend;         // [N]
  int32_t* level_nodes;  // [N] inner node ids grouped by depth
  int64_t level_off[msp::kMaxDepth + 2];   // runs of level_nodes (inner nodes only)
  msp::NodeRec* rec[2];  // [N + 1] per type (index N: zero sentinel, never visited)
  int32_t* vs[2];        // [n] per type: counts in sorted order (bucket members)
  int32_t* err;          // [1] sticky device error flags
  bool refreshed;
  bool inside;           // every position lies in the closed cube, and the cube lies
                         // within 2^18 edges of the origin
  void* slab_n;          // one allocation holding the neuron arrays ...
  void* slab_N;          // ... and one holding the node arrays
};

#define MSP_HIP_TRY(expr)                                   \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) {                                 \
      (void)hipGetLastError();                              \
      return e_ == hipErrorOutOfMemory ? MSP_ERR_OOM : MSP_ERR_HIP; \
    }                                                       \
  } while (0)

namespace msp {

// Registry of the live handles the library has handed out (octrees, batch plans and
// update cycles).
// A handle is valid exactly while it is registered: every entry point looks the
// pointer up here instead of reading through it, so a freed, foreign or doubly freed
// handle is rejected without touching freed memory. (A handle whose address a later
// build or plan has reused names that new object.)
enum class HandleKind : int { kOctree = 1, kBatch = 2, kCycle = 3 };

inline std::mutex& handle_mutex() {
  static std::mutex m;
  return m;
}

inline std::unordered_map<const void*, HandleKind>& live_handles() {
  static std::unordered_map<const void*, HandleKind> h;
  return h;
}

inline void handle_register(const void* p, HandleKind k) {
  std::lock_guard<std::mutex> g(handle_mutex());
  live_handles()[p] = k;
}

inline bool handle_live(const void* p, HandleKind k) {
  if (!p) return false;
  std::lock_guard<std::mutex> g(handle_mutex());
  const auto it = live_handles().find(p);
  return it != live_handles().end() && it->second == k;
}

// Unregister p if it is a live handle of kind k; true if it was (exactly one of two
// concurrent frees of one handle gets true).
inline bool handle_take(const void* p, HandleKind k) {
  if (!p) return false;
  std::lock_guard<std::mutex> g(handle_mutex());
  const auto it = live_handles().find(p);
  if (it == live_handles().end() || it->second != k) return false;
  live_handles().erase(it);
  return true;
}

inline bool handle_ok(const msp_octree_s* t) { return handle_live(t, HandleKind::kOctree); }

// The library's own stream-ordered memory pool on `device`: memory freed to it stays
// mapped for the next allocation (release threshold = unlimited), so the per-call
// temporaries of large updates do not pay for page mapping on every call. Other users
// of the device's default pool are not affected.
inline hipError_t lib_pool(int device, hipMemPool_t* out) {
  static std::mutex m;
  static hipMemPool_t pools[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(m);
  if (!pools[device]) {
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    hipMemPool_t pool = nullptr;
    hipError_t e = hipMemPoolCreate(&pool, &props);
    if (e != hipSuccess) return e;
    uint64_t keep = ~(uint64_t)0;
    e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    if (e != hipSuccess) {
      (void)hipMemPoolDestroy(pool);
      return e;
    }
    pools[device] = pool;
  }
  *out = pools[device];
  return hipSuccess;
}

// A non-blocking stream of the library's own on `device` (default priority), on which
// memory whose users have all finished is returned to the pool.
inline hipError_t lib_stream(int device, hipStream_t* out) {
  static std::mutex m;
  static hipStream_t streams[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(m);
  if (!streams[device]) {
    hipError_t e = hipStreamCreateWithFlags(&streams[device], hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  *out = streams[device];
  return hipSuccess;
}

// `bytes` of device memory from the library pool, ordered on stream `s` (current device).
inline hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  hipMemPool_t pool;
  if ((e = lib_pool(dev, &pool)) != hipSuccess) return e;
  return hipMallocFromPoolAsync(p, bytes == 0 ? 256 : bytes, pool, s);
}

// Stream-ordered temporary device memory; released on the same stream.
struct Temp {
  hipStream_t s;
  void* p = nullptr;
  explicit Temp(hipStream_t st) : s(st) {}
  hipError_t alloc(size_t bytes) { return pool_alloc(&p, bytes, s); }
  ~Temp() {
    if (p) (void)hipFreeAsync(p, s);
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  return (unsigned)g;
}

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Carves 256-byte aligned arrays out of one allocation (base null: only sizes it).
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(int64_t count) {
    T* q = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += align_up(sizeof(T) * (size_t)(count > 0 ? count : 1));
    return q;
  }
  void* take_bytes(size_t bytes) {
    void* q = base ? base + off : nullptr;
    off += align_up(bytes);
    return q;
  }
};

__global__ void fill_i32_k(int32_t* p, int64_t n, int32_t v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

__global__ void fill_i64_k(int64_t* p, int64_t n, int64_t v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

__global__ void copy_i32_k(const int32_t* __restrict__ from, int32_t* __restrict__ to, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) to[k] = from[k];
}

// An item count known on the host (p null: v) or only on the device (*p, clamped to
// [0, v]: the launch is sized for the bound v and threads past the count return).
// Device counts let a sequence of launches run without reading anything back, so that
// it can be enqueued ahead and captured in a graph.
struct DevCount {
  int64_t v;
  const int64_t* p;
  __device__ __forceinline__ int64_t get() const {
    if (!p) return v;
    const int64_t c = *p;
    return c < 0 ? 0 : (c < v ? c : v);
  }
};

inline DevCount host_count(int64_t n) { return DevCount{n, nullptr}; }

// Launches over a device count are sized for its bound but hold at most kStrideGrid
// blocks (one full residency of the chip at 256 threads); their threads stride over
// the items.
constexpr unsigned kStrideGrid = 2048;

inline unsigned grid_cap(int64_t n, int block) {
  const unsigned g = grid_for(n, block);
  return g < kStrideGrid ? g : kStrideGrid;
}

__device__ __forceinline__ int64_t gtid() {
  return (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

// A step number given by value, or read on the device (p non-null).
struct DevStep {
  uint64_t v;
  const uint64_t* p;
  __device__ __forceinline__ uint64_t get() const { return p ? *p : v; }
};

inline DevStep host_step(uint64_t step) { return DevStep{step, nullptr}; }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 64x64->128-bit products and a xor with the round key; the key advances by the
// Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2,
                                              uint64_t& c3, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t a0 = 0xD2E7470EE14C6C93ULL * c0;
    const uint64_t h0 = __umul64hi(0xD2E7470EE14C6C93ULL, c0);
    const uint64_t a1 = 0xCA5A826395121157ULL * c2;
    const uint64_t h1 = __umul64hi(0xCA5A826395121157ULL, c2);
    const uint64_t n0 = h1 ^ c1 ^ k0;
    const uint64_t n2 = h0 ^ c3 ^ k1;
    c0 = n0;
    c1 = a1;
    c2 = n2;
    c3 = a0;
    k0 += 0x9E3779B97F4A7C15ULL;
    k1 += 0xBB67AE8584CAA73BULL;
  }
}

__device__ __forceinline__ uint64_t philox_word0(uint64_t seed, uint64_t stream, uint64_t a,
                                                 uint64_t b, uint64_t c, uint64_t d) {
  philox4x64_10(a, b, c, d, seed, stream);
  return a;
}

}  // namespace msp
