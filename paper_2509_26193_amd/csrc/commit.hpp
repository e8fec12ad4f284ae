// Request acceptance (Sec. III-A, "Update of synapses"; Sec. III-B: all requests
// are formed before they are exchanged, accepted locally and answered yes/no).
// Requests on one (target, type) pair form a group; the group accepts the
// min(requests, vacancies) requests of smallest Philox priority, ties by (i, j).
// The result does not depend on the order in which requests are grouped.
#pragma once

#include "common.hpp"

namespace msp {

constexpr int kCommitBlock = 256;
constexpr int32_t kCommitCapacity = 1;      // more accepted requests than list capacity
constexpr int32_t kSmallGroup = 8;          // groups up to this size are ranked by one thread

// A group's decision for its members: all accepted, none, those up to a (priority,
// slot) threshold (the v-th smallest), or, for groups above kSmallGroup requests,
// ranked per request.
enum : int32_t { kGroupAll = 0, kGroupNone = 1, kGroupThr = 2, kGroupRank = 3 };
struct GroupThr {
  uint64_t prio;
  int32_t slot;
  int32_t mode;
};

// Source of every request slot below S.
__global__ void __launch_bounds__(kCommitBlock) src_of_k(const int64_t* __restrict__ off, int64_t n,
                                                        DevCount S, int32_t* __restrict__ src_of) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t S_ = S.get();
  const int64_t e = off[i + 1] < S_ ? off[i + 1] : S_;
  for (int64_t s = off[i]; s < e; ++s) src_of[s] = (int32_t)i;
}

// The launches over the S requests below are sized by grid_cap and stride over them.

// Group key 2g + type, priority, and the per-group request count.
__global__ void __launch_bounds__(kCommitBlock) req_key_k(
    const int32_t* __restrict__ target, const int64_t* __restrict__ off,
    const int32_t* __restrict__ src_of, const uint8_t* __restrict__ type, DevCount S, int64_t n,
    uint64_t seed, DevStep step, int64_t* __restrict__ key, uint64_t* __restrict__ prio,
    int32_t* __restrict__ cnt, int32_t* __restrict__ within, int32_t* err) {
  const int64_t S_ = S.get();
  const uint64_t st = step.get();
  for (int64_t s = gtid(); s < S_; s += gstride()) {
    const int32_t g = target[s];
    const int32_t i = src_of[s];
    if (g < 0 || g >= n) {
      if (g >= n) atomicOr(err, kErrArgs);
      key[s] = -1;
      continue;
    }
    const int64_t k = 2 * (int64_t)g + (type[i] ? 1 : 0);
    key[s] = k;
    prio[s] = philox_word0(seed, 1, (uint64_t)i, (uint64_t)(s - off[i]), st, 0);
    within[s] = atomicAdd(&cnt[k], 1);      // the request's place in its group
  }
}

// Each request at its group's offset plus its place in the group (the order within a
// group is the counting atomics' order; the decisions below do not depend on it).
__global__ void __launch_bounds__(kCommitBlock) req_scatter_k(const int64_t* __restrict__ key,
                                                             DevCount S,
                                                             const int32_t* __restrict__ seg_off,
                                                             const int32_t* __restrict__ within,
                                                             int32_t* __restrict__ seg) {
  const int64_t S_ = S.get();
  for (int64_t s = gtid(); s < S_; s += gstride()) {
    const int64_t k = key[s];
    if (k < 0) continue;
    seg[seg_off[k] + within[s]] = (int32_t)s;
  }
}

// One thread per group k (target k / 2, type k % 2; its requests seg[lo, hi)), the
// group's offsets and vacancies read in order: its accepted count min(requests,
// vacancies) into acc_cnt[k] and its decision into thr[k]. Where some but not all are
// accepted (and the group has at most kSmallGroup requests), the threshold is the
// (priority, slot) of the member that exactly v - 1 others precede.
__global__ void __launch_bounds__(kCommitBlock) group_thr_k(
    const uint64_t* __restrict__ prio, const int32_t* __restrict__ seg_off,
    const int32_t* __restrict__ seg, int64_t n2, const int32_t* __restrict__ vexc,
    const int32_t* __restrict__ vinh, GroupThr* __restrict__ thr, int32_t* __restrict__ acc_cnt) {
  for (int64_t k = gtid(); k < n2; k += gstride()) {
    const int32_t lo = seg_off[k], hi = seg_off[k + 1];
    const int32_t c = hi - lo;
    if (c == 0) {
      acc_cnt[k] = 0;
      continue;
    }
    const int32_t g = (int32_t)(k >> 1);
    int32_t v = (k & 1) ? vinh[g] : vexc[g];
    v = v < 0 ? 0 : v;
    acc_cnt[k] = c < v ? c : v;
    GroupThr t{0, 0, c <= v ? kGroupAll : v == 0 ? kGroupNone : kGroupRank};
    if (t.mode == kGroupRank && c <= kSmallGroup) {
      // the members' slots and priorities in registers first (independent loads), then
      // every member ranked against the others
      int32_t ms[kSmallGroup];
      uint64_t mp[kSmallGroup];
#pragma unroll
      for (int r = 0; r < kSmallGroup; ++r) ms[r] = r < c ? seg[lo + r] : 0;
#pragma unroll
      for (int r = 0; r < kSmallGroup; ++r) mp[r] = r < c ? prio[ms[r]] : 0;
#pragma unroll
      for (int q = 0; q < kSmallGroup; ++q) {
        int32_t rank = 0;
#pragma unroll
        for (int r = 0; r < kSmallGroup; ++r)
          rank += (r < c && (mp[r] < mp[q] || (mp[r] == mp[q] && ms[r] < ms[q]))) ? 1 : 0;
        if (q < c && rank == v - 1) t = GroupThr{mp[q], ms[q], kGroupThr};
      }
    }
    thr[k] = t;
  }
}

// Accept iff fewer than v requests of the group precede this one in (prio, i, j) order.
// Slots s are in (i, j) order, so (i, j) ties compare as slot indices.
__device__ __forceinline__ uint8_t rank_accept(const int64_t* __restrict__ key,
                                               const uint64_t* __restrict__ prio,
                                               const int32_t* __restrict__ seg_off,
                                               const int32_t* __restrict__ seg,
                                               const int32_t* __restrict__ vexc,
                                               const int32_t* __restrict__ vinh, int64_t s) {
  const int64_t k = key[s];
  if (k < 0) return 0;
  const int32_t g = (int32_t)(k >> 1);
  int32_t v = (k & 1) ? vinh[g] : vexc[g];
  v = v < 0 ? 0 : v;
  const int32_t lo = seg_off[k], hi = seg_off[k + 1];
  if (hi - lo <= v) return 1;
  const uint64_t ps = prio[s];
  int32_t rank = 0;
  for (int32_t q = lo; q < hi && rank < v; ++q) {
    const int32_t o = seg[q];
    const uint64_t po = prio[o];
    rank += (po < ps || (po == ps && o < s)) ? 1 : 0;
  }
  return rank < v ? 1 : 0;
}

// Each request's decision from its group's (one gather per request; the members of
// groups above kSmallGroup requests are ranked here, one thread per request).
__global__ void __launch_bounds__(kCommitBlock) req_decide_k(
    const int64_t* __restrict__ key, const uint64_t* __restrict__ prio,
    const GroupThr* __restrict__ thr, const int32_t* __restrict__ seg_off,
    const int32_t* __restrict__ seg, DevCount S, const int32_t* __restrict__ vexc,
    const int32_t* __restrict__ vinh, uint8_t* __restrict__ acc) {
  const int64_t S_ = S.get();
  for (int64_t s = gtid(); s < S_; s += gstride()) {
    const int64_t k = key[s];
    uint8_t a = 0;
    if (k >= 0) {
      const GroupThr t = thr[k];
      if (t.mode == kGroupAll) {
        a = 1;
      } else if (t.mode == kGroupThr) {
        const uint64_t ps = prio[s];
        a = (ps < t.prio || (ps == t.prio && s <= t.slot)) ? 1 : 0;
      } else if (t.mode == kGroupRank) {
        a = rank_accept(key, prio, seg_off, seg, vexc, vinh, s);
      }
    }
    acc[s] = a;
  }
}

// Writes the accepted requests' synapses at their places in the output list, unless
// the list (capacity `cap`) cannot hold them all or a target was out of range
// (kErrArgs in *flags): then it writes nothing (and sets kCommitCapacity for the
// former). The vacancies are taken by dec_groups_k and dec_sources_k under the same
// condition.
__device__ __forceinline__ bool commit_ok(const int64_t* __restrict__ dst, int64_t S_, int64_t cap,
                                          const int32_t* flags) {
  return S_ > 0 && !(*flags & kErrArgs) && dst[S_] <= cap;
}

__global__ void __launch_bounds__(kCommitBlock) commit_write_k(
    const uint8_t* __restrict__ acc, const int64_t* __restrict__ dst, const int64_t* __restrict__ key,
    const int32_t* __restrict__ src_of, DevCount S, int64_t cap, int32_t* syn_src, int32_t* syn_tgt,
    uint8_t* syn_type, uint8_t* acc_out, int32_t* flags) {
  const int64_t S_ = S.get();
  if (S_ == 0 || (*flags & kErrArgs)) return;
  if (dst[S_] > cap) {
    if (gtid() == 0) atomicOr(flags, kCommitCapacity);
    return;
  }
  for (int64_t s = gtid(); s < S_; s += gstride()) {
    const uint8_t a = acc[s];
    if (acc_out) acc_out[s] = a;
    if (!a) continue;
    const int64_t k = key[s];
    const int32_t g = (int32_t)(k >> 1);
    const int ty = (int)(k & 1);
    const int64_t p = dst[s];
    syn_src[p] = src_of[s];
    syn_tgt[p] = g;
    syn_type[p] = (uint8_t)ty;
  }
}

// Each group's accepted count off its target's vacancies of that type (the two types
// of a target are different arrays, so no two threads write one count).
__global__ void __launch_bounds__(kCommitBlock) dec_groups_k(
    const int32_t* __restrict__ acc_cnt, int64_t n2, const int64_t* __restrict__ dst, DevCount S,
    int64_t cap, const int32_t* flags, int32_t* __restrict__ vexc, int32_t* __restrict__ vinh) {
  if (!commit_ok(dst, S.get(), cap, flags)) return;
  for (int64_t k = gtid(); k < n2; k += gstride()) {
    const int32_t a = acc_cnt[k];
    if (a) ((k & 1) ? vinh : vexc)[k >> 1] -= a;
  }
}

// Each source's accepted requests off its vacant axonal elements.
__global__ void __launch_bounds__(kCommitBlock) dec_sources_k(
    const int64_t* __restrict__ off, int64_t n, const uint8_t* __restrict__ acc,
    const int64_t* __restrict__ dst, DevCount S, int64_t cap, const int32_t* flags,
    int32_t* __restrict__ vac_axon) {
  const int64_t S_ = S.get();
  if (!commit_ok(dst, S_, cap, flags)) return;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const int64_t e = off[i + 1] < S_ ? off[i + 1] : S_;
    int32_t a = 0;
    for (int64_t s = off[i]; s < e; ++s) a += acc[s];
    if (a) vac_axon[i] -= a;
  }
}

struct AccFlag {
  __device__ int64_t operator()(uint8_t a, int64_t) const { return (int64_t)a; }
};

// Synapses formed: the accepted requests, or 0 where commit_write_k wrote nothing.
__global__ void formed_k(const int64_t* __restrict__ dst, DevCount S, int64_t cap,
                         const int32_t* __restrict__ flags, int64_t* __restrict__ n_formed) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t S_ = S.get();
  const int64_t f = S_ == 0 ? 0 : dst[S_];
  *n_formed = ((*flags & kErrArgs) || f > cap) ? 0 : f;
}

__global__ void copy_scalar_k(const int64_t* __restrict__ src, int64_t* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

}  // namespace msp
