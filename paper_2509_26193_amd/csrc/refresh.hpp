// Vacancy refresh (Sec. III-B, "Division of work"): the leaves in one pass, then the
// inner nodes bottom-up, one launch per depth.
// A leaf takes its neuron's count and position; an inner node the sum of its
// children's counts and the count-weighted mean of their centroids, accumulated in
// float64 left to right in octant order with one rounding per operation (the
// library is compiled without FP contraction, so no product is fused into a sum).
#pragma once

#include "common.hpp"

namespace msp {

constexpr int kRefreshBlock = 256;

struct Acc3 {
  int64_t v = 0;
  double x = 0.0, y = 0.0, z = 0.0;
  __device__ __forceinline__ void add(int64_t vk, double cx, double cy, double cz) {
    v += vk;
    if (vk > 0) {
      const double w = (double)vk;
      x = x + w * cx;
      y = y + w * cy;
      z = z + w * cz;
    }
  }
  __device__ __forceinline__ void store(NodeRec& r, int32_t* err) const {
    if (v > 0x7FFFFFFF) atomicOr(err, kErrOverflow);
    r.v = (int32_t)v;
    if (v > 0) {
      const double d = (double)v;
      r.x = x / d;
      r.y = y / d;
      r.z = z / d;
    } else {
      r.x = r.y = r.z = 0.0;
    }
  }
};

// Leaves, one thread per neuron in sorted order (leaf indices, records and member
// counts are read and written in order; positions and the caller's vacancy arrays
// are gathered by id). A bucket leaf is done by its first member's thread, its
// members in sorted order (id order within the finest cell).
__global__ void __launch_bounds__(kRefreshBlock) refresh_leaves_k(
    int64_t n, NodeRec* __restrict__ r0, NodeRec* __restrict__ r1,
    const int32_t* __restrict__ leaf_at, const int32_t* __restrict__ nbeg,
    const int32_t* __restrict__ nend, const int32_t* __restrict__ order,
    const double* __restrict__ pos, const int32_t* __restrict__ vexc,
    const int32_t* __restrict__ vinh, int32_t* __restrict__ vs0, int32_t* __restrict__ vs1,
    int32_t* err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t x = leaf_at[p];
  const uint32_t meta = r0[x].meta;
  if (!(meta & kBucketBit)) {
    const int32_t id = order[p];
    const int32_t a = vexc[id], b = vinh[id];
    if (a < 0 || b < 0) atomicOr(err, kErrNegative);
    NodeRec e, f;
    e.x = f.x = pos[3 * (int64_t)id];
    e.y = f.y = pos[3 * (int64_t)id + 1];
    e.z = f.z = pos[3 * (int64_t)id + 2];
    e.v = a < 0 ? 0 : a;
    f.v = b < 0 ? 0 : b;
    e.meta = f.meta = meta;
    r0[x] = e;
    r1[x] = f;
    vs0[p] = e.v;
    vs1[p] = f.v;
    return;
  }
  if (p != nbeg[x]) return;
  Acc3 A, B;
  for (int32_t q = nbeg[x]; q < nend[x]; ++q) {
    const int32_t id = order[q];
    int32_t a = vexc[id], b = vinh[id];
    if (a < 0 || b < 0) atomicOr(err, kErrNegative);
    a = a < 0 ? 0 : a;
    b = b < 0 ? 0 : b;
    const double px = pos[3 * (int64_t)id], py = pos[3 * (int64_t)id + 1],
                 pz = pos[3 * (int64_t)id + 2];
    A.add(a, px, py, pz);
    B.add(b, px, py, pz);
    vs0[q] = a;
    vs1[q] = b;
  }
  NodeRec e, f;
  e.meta = f.meta = meta;
  A.store(e, err);
  B.store(f, err);
  r0[x] = e;
  r1[x] = f;
}

// Inner nodes of one depth (after every deeper depth and the leaves).
__global__ void __launch_bounds__(kRefreshBlock) refresh_level_k(
    const int32_t* __restrict__ nodes, int64_t cnt, NodeRec* __restrict__ r0,
    NodeRec* __restrict__ r1, int32_t* err) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cnt) return;
  const int32_t x = nodes[q];
  const uint32_t meta = r0[x].meta;
  // children are x+1, then each child's subtree end, up to our own end
  const int32_t end = (int32_t)(meta & kSkipMask);
  Acc3 A, B;
  int32_t c = x + 1;
  while (c < end) {
    const NodeRec ca = r0[c];
    const NodeRec cb = r1[c];
    A.add(ca.v, ca.x, ca.y, ca.z);
    B.add(cb.v, cb.x, cb.y, cb.z);
    c = (ca.meta & kLeafBit) ? c + 1 : (int32_t)(ca.meta & kSkipMask);
  }
  NodeRec e, f;
  e.meta = f.meta = meta;
  A.store(e, err);
  B.store(f, err);
  r0[x] = e;
  r1[x] = f;
}

}  // namespace msp
