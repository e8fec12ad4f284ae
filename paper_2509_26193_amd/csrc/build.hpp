// Octree construction (Sec. III-B, "Spatial octree"): Morton keys, sort, and the
// node topology in depth-first pre-order, derived from adjacent common prefixes.
#pragma once

#include "common.hpp"
#include "scan.hpp"

namespace msp {

constexpr int kBuildBlock = 256;

// Quantise each axis to 21 bits and interleave: digit k (1..21, most significant
// first) = 4*x_bit + 2*y_bit + z_bit of bit (21-k). Non-finite positions raise a flag.
__device__ __forceinline__ uint64_t spread3(uint64_t v) {   // 21 bits -> every third bit
  v &= 0x1FFFFFull;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__device__ __forceinline__ uint64_t quantise(double x, double lo, double edge) {
  double f = floor(((x - lo) / edge) * 2097152.0);
  f = (f >= 0.0) ? f : 0.0;
  f = (f > 2097151.0) ? 2097151.0 : f;
  return (uint64_t)f;
}

__global__ void __launch_bounds__(kBuildBlock) keys_k(const double* __restrict__ pos_in, int64_t n,
                                                     double x0, double y0, double z0, double edge,
                                                     double* __restrict__ pos, uint64_t* keys,
                                                     int32_t* ids, int32_t* err,
                                                     int32_t* outside) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = pos_in[3 * i + 0], y = pos_in[3 * i + 1], z = pos_in[3 * i + 2];
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) atomicOr(err, kErrNonFinite);
  // a position outside the closed cube (it is clamped into an edge cell); one atomic
  // per wave at most
  const bool out = !(x >= x0 && x <= x0 + edge && y >= y0 && y <= y0 + edge && z >= z0 &&
                     z <= z0 + edge);
  const uint64_t outs = __ballot(out);
  if (outs && (threadIdx.x & 63) == (unsigned)(__ffsll((unsigned long long)outs) - 1))
    atomicOr(outside, 1);
  pos[3 * i + 0] = x;
  pos[3 * i + 1] = y;
  pos[3 * i + 2] = z;
  const uint64_t qx = quantise(x, x0, edge), qy = quantise(y, y0, edge), qz = quantise(z, z0, edge);
  keys[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
  ids[i] = (int32_t)i;
}

// Number of equal leading octant digits of two 63-bit keys (21 if equal).
__device__ __forceinline__ int common_digits(uint64_t a, uint64_t b) {
  const uint64_t x = a ^ b;
  if (x == 0) return kMaxDepth;
  return (__clzll((long long)x) - 1) / 3;
}

// Node (start m, depth k) exists for k in [k_lo(m), k_hi(m)] with
// k_lo = cl + 1 and k_hi = min(21, max(cl, cr) + 1), where cl / cr are the common digit
// counts with the left / right neighbour in sorted order (-1 at the ends). Pre-order
// numbering: node index = (nodes starting before m) + (k - k_lo).
__global__ void __launch_bounds__(kBuildBlock) node_count_k(const uint64_t* __restrict__ keys,
                                                           int64_t n, int32_t* cnt) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const int cl = m == 0 ? -1 : common_digits(keys[m - 1], keys[m]);
  const int cr = m == n - 1 ? -1 : common_digits(keys[m], keys[m + 1]);
  const int klo = cl + 1;
  const int khi = min(kMaxDepth, max(cl, cr) + 1);
  cnt[m] = khi >= klo ? khi - klo + 1 : 0;
}

__device__ __forceinline__ uint64_t prefix_of(uint64_t key, int k) {
  return k == 0 ? 0ull : key >> (3 * (kMaxDepth - k));
}

__global__ void __launch_bounds__(kBuildBlock) nodes_k(const uint64_t* __restrict__ keys,
                                                      const int32_t* __restrict__ order, int64_t n,
                                                      const int32_t* __restrict__ base,
                                                      int32_t* skip, uint8_t* depth, int32_t* nbeg,
                                                      int32_t* nend, int32_t* leaf_of,
                                                      int32_t* leaf_at) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const int cl = m == 0 ? -1 : common_digits(keys[m - 1], keys[m]);
  const int cr = m == n - 1 ? -1 : common_digits(keys[m], keys[m + 1]);
  const int klo = cl + 1;
  const int khi = min(kMaxDepth, max(cl, cr) + 1);
  if (khi < klo) return;
  const uint64_t km = keys[m];
  int64_t end = m + 1;              // ranges grow as the depth decreases
  for (int k = khi; k >= klo; --k) {
    int64_t e;
    if (k == 0) {
      e = n;
    } else {
      const uint64_t P = prefix_of(km, k);
      if (end >= n || prefix_of(keys[end], k) != P) {
        e = end;
      } else {                     // gallop then bisect for the first key outside the cell
        int64_t lo = end, step = 1;
        while (lo + step < n && prefix_of(keys[lo + step], k) == P) {
          lo += step;
          step <<= 1;
        }
        int64_t hi = lo + step < n ? lo + step : n;
        while (hi - lo > 1) {
          const int64_t mid = lo + (hi - lo) / 2;
          if (prefix_of(keys[mid], k) == P) lo = mid; else hi = mid;
        }
        e = hi;
      }
    }
    end = e;
    const int64_t idx = (int64_t)base[m] + (k - klo);
    skip[idx] = base[e];
    depth[idx] = (uint8_t)k;
    nbeg[idx] = (int32_t)m;
    nend[idx] = (int32_t)e;
    const bool leaf = (e - m == 1) || k == kMaxDepth;
    if (leaf)
      for (int64_t p = m; p < e; ++p) {
        leaf_of[order[p]] = (int32_t)idx;
        leaf_at[p] = (int32_t)idx;
      }
  }
}

// Lanes of the wave holding the same depth as this lane (5-bit values; inactive
// lanes and lanes with d < 0 are excluded).
__device__ __forceinline__ uint64_t same_depth_lanes(int d) {
  uint64_t peers = __ballot(d >= 0);
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const bool bit = (d >> b) & 1;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Nodes per block of the per-depth passes: enough that the per-block global atomics
// (one per depth) do not queue up on the few hot depth counters.
constexpr int kLevelItems = 16;

// Inner nodes per depth (leaves are refreshed in sorted order, not by depth): one LDS
// atomic per distinct depth and wave, one global atomic per depth and block of
// kBuildBlock * kLevelItems nodes. A leaf is a node whose subtree ends right after it.
__device__ __forceinline__ int inner_depth(const uint8_t* depth, const int32_t* skip, int64_t x,
                                           int64_t N) {
  return (x < N && skip[x] != (int32_t)(x + 1)) ? (int)depth[x] : -1;
}

__global__ void __launch_bounds__(kBuildBlock) level_count_k(const uint8_t* __restrict__ depth,
                                                            const int32_t* __restrict__ skip,
                                                            int64_t N, int32_t* level_cnt) {
  __shared__ int32_t c[kMaxDepth + 1];
  if (threadIdx.x <= kMaxDepth) c[threadIdx.x] = 0;
  __syncthreads();
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int64_t base = (int64_t)blockIdx.x * kBuildBlock * kLevelItems + threadIdx.x;
  for (int k = 0; k < kLevelItems; ++k) {
    const int64_t x = base + (int64_t)k * kBuildBlock;
    const int d = inner_depth(depth, skip, x, N);
    const uint64_t peers = same_depth_lanes(d);
    if (d >= 0 && lane == __ffsll((unsigned long long)peers) - 1) atomicAdd(&c[d], __popcll(peers));
  }
  __syncthreads();
  if (threadIdx.x <= kMaxDepth && c[threadIdx.x]) atomicAdd(&level_cnt[threadIdx.x], c[threadIdx.x]);
}

// Group inner node ids by depth (order within a depth is arbitrary: the refresh of one
// depth treats its nodes independently). Same blocking as level_count_k.
__global__ void __launch_bounds__(kBuildBlock) level_scatter_k(const uint8_t* __restrict__ depth,
                                                              const int32_t* __restrict__ skip,
                                                              int64_t N, int32_t* cursor,
                                                              int32_t* level_nodes) {
  __shared__ int32_t c[kMaxDepth + 1];
  __shared__ int32_t base_d[kMaxDepth + 1];
  if (threadIdx.x <= kMaxDepth) c[threadIdx.x] = 0;
  __syncthreads();
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const int64_t base = (int64_t)blockIdx.x * kBuildBlock * kLevelItems + threadIdx.x;
  int d[kLevelItems];
  int r[kLevelItems];
#pragma unroll
  for (int k = 0; k < kLevelItems; ++k) {
    const int64_t x = base + (int64_t)k * kBuildBlock;
    d[k] = inner_depth(depth, skip, x, N);
    const uint64_t peers = same_depth_lanes(d[k]);
    const int leader = __ffsll((unsigned long long)peers) - 1;
    int r0 = 0;
    if (d[k] >= 0 && lane == leader) r0 = atomicAdd(&c[d[k]], __popcll(peers));
    r[k] = __shfl(r0, leader < 0 ? 0 : leader, kWave) + __popcll(peers & ((1ull << lane) - 1ull));
  }
  __syncthreads();
  if (threadIdx.x <= kMaxDepth && c[threadIdx.x])
    base_d[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], c[threadIdx.x]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kLevelItems; ++k)
    if (d[k] >= 0) level_nodes[base_d[d[k]] + r[k]] = (int32_t)(base + (int64_t)k * kBuildBlock);
}

// Start of each depth's run in level_nodes: the exclusive prefix of the per-depth
// counts (one thread; kMaxDepth + 1 values).
__global__ void level_cursor_k(const int32_t* __restrict__ counts, int32_t* __restrict__ cursor) {
  int32_t acc = 0;
  for (int k = 0; k <= kMaxDepth; ++k) {
    cursor[k] = acc;
    acc += counts[k];
  }
}

// Per-type records start with count 0 and the node's meta word: an inner node keeps
// its subtree end and depth, a leaf its neuron id, a bucket leaf its own index.
__global__ void __launch_bounds__(kBuildBlock) init_meta_k(const int32_t* __restrict__ skip,
                                                          const uint8_t* __restrict__ depth,
                                                          const int32_t* __restrict__ nbeg,
                                                          const int32_t* __restrict__ nend,
                                                          const int32_t* __restrict__ order,
                                                          int64_t N, NodeRec* r0, NodeRec* r1) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  const int32_t sk = skip[x];
  uint32_t meta;
  if (sk != x + 1)
    meta = ((uint32_t)sk & kSkipMask) | ((uint32_t)depth[x] << kSkipBits);
  else if (nend[x] - nbeg[x] == 1)
    meta = kLeafBit | (uint32_t)order[nbeg[x]];
  else
    meta = kLeafBit | kBucketBit | (uint32_t)x;
  NodeRec r;
  r.x = r.y = r.z = 0.0;
  r.v = 0;
  r.meta = meta;
  r0[x] = r;
  r1[x] = r;
}

}  // namespace msp
