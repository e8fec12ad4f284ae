// The change of the network between two connectivity updates (Sec. III-A, "Update of
// synaptic elements" and the first sub-phase of "Update of synapses"), on the device:
//   * growth: per neuron j and element kind k (0 axon, 1 excitatory dendrite,
//     2 inhibitory dendrite) a calcium value Ca ~ N(mean, sd) (Box-Muller on Philox
//     words 0 and 1, key (seed, 2), counter (j, k, step, 0)) moves the continuous
//     element count by dz = steps * nu * (2 exp(-((Ca - xi) / zeta)^2) - 1), with
//     xi = (eta + eps) / 2 and zeta = (eps - eta) / (2 sqrt(ln 2)); z = max(z + dz, 0);
//   * deletion: the round(frac * m) synapses of smallest (Philox word 0, key (seed, 3),
//     counter (s, step, 0, 0); then s) go, s being the place in the list at the start
//     of the step;
//   * retraction, for k = 0, 1, 2 in turn: a neuron whose floor(z) fell below its
//     bound elements of kind k loses that many of its synapses of that kind, those of
//     smallest (top 32 bits of Philox word 0, key (seed, 4), counter (s, step, k, 0);
//     then s);
//   * a synapse (i, g, type) binds one axonal element of i and one dendritic element
//     of kind 1 + type of g; breaking it frees both; the list keeps its order;
//   * vacant elements: floor(z) - bound.
// Selections are sorts of 64-bit keys (priority, or owner and priority) with the
// synapse index as a stable tie-break, so every choice is exact and reproducible.
#pragma once

#include "scan.hpp"

namespace msp {

constexpr int kPlastBlock = 256;

struct SynList {
  int32_t* src;
  int32_t* tgt;
  uint8_t* type;
};

__global__ void __launch_bounds__(kPlastBlock) growth_k(double* __restrict__ z, int64_t n,
                                                       uint64_t seed, DevStep step,
                                                       double ca_mean, double ca_sd, double xi,
                                                       double zeta, double scale) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 3 * n) return;
  const int64_t k = g / n, j = g - k * n;
  uint64_t c0 = (uint64_t)j, c1 = (uint64_t)k, c2 = step.get(), c3 = 0;
  philox4x64_10(c0, c1, c2, c3, seed, 2);
  const double u1 = (double)((c0 >> 11) + 1) * 0x1p-53;     // (0, 1]
  const double u2 = (double)(c1 >> 11) * 0x1p-53;           // [0, 1)
  const double two_pi = 6.283185307179586476925286766559;
  const double gauss = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
  const double ca = ca_mean + ca_sd * gauss;
  const double r = (ca - xi) / zeta;
  const double e = exp(-(r * r));
  const double zz = z[g] + scale * (2.0 * e - 1.0);
  z[g] = zz > 0.0 ? zz : 0.0;
}

// Frees the two elements a synapse binds.
__device__ __forceinline__ void unbind(const SynList& L, int64_t s, int64_t n, int32_t* bound) {
  atomicSub(&bound[L.src[s]], 1);
  atomicSub(&bound[(1 + (int64_t)L.type[s]) * n + L.tgt[s]], 1);
}

__global__ void __launch_bounds__(kPlastBlock) del_keys_k(uint64_t* __restrict__ key,
                                                         int32_t* __restrict__ val, DevCount m,
                                                         uint64_t seed, DevStep step) {
  const int64_t m_ = m.get();
  const uint64_t st = step.get();
  for (int64_t s = gtid(); s < m_; s += gstride()) {
    key[s] = philox_word0(seed, 3, (uint64_t)s, st, 0, 0);
    val[s] = (int32_t)s;
  }
}

// Deletion as a selection, not a sort: the `want` synapses of smallest (priority,
// index) go. Most significant digit first, each pass narrows the candidates to the
// keys that share the digits chosen so far, and counts the candidates' next digit.
struct DelSelect {
  uint64_t prefix;              // digits chosen so far (the threshold key, at the end)
  uint64_t mask;                // their bits
  int64_t want;                 // synapses still to choose among the candidates
};

// Synapses a deletion removes from a list of m: round(frac m), halves up, at most m
// (the product and the sum rounded separately, as on the host).
__host__ __device__ inline int64_t delete_count(double frac, int64_t m) {
#pragma clang fp contract(off)
  const double w = floor(frac * (double)m + 0.5);
  const int64_t c = (int64_t)w;
  return c < m ? c : m;
}

__global__ void del_select_init_k(DelSelect* st, double frac, DevCount m, uint32_t* hist) {
  if (threadIdx.x == 0) {
    st->prefix = 0;
    st->mask = 0;
    st->want = delete_count(frac, m.get());
  }
  hist[threadIdx.x] = 0;        // 256 threads
}

// Histogram of digit (key >> shift) & 255 over the keys that match the chosen digits.
__global__ void __launch_bounds__(kPlastBlock) del_select_hist_k(const uint64_t* __restrict__ key,
                                                                DevCount mc, const DelSelect* st,
                                                                int shift, uint32_t* hist) {
  __shared__ uint32_t h[256];
  for (int d = threadIdx.x; d < 256; d += blockDim.x) h[d] = 0;
  __syncthreads();
  const uint64_t prefix = st->prefix, mask = st->mask;
  const int64_t m = st->want > 0 ? mc.get() : 0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < m;
       s += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = key[s];
    if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += blockDim.x)
    if (h[d]) atomicAdd(&hist[d], h[d]);
}

// One block of 256 threads: the digit whose candidates hold the want-th smallest key;
// the candidates with smaller digits are all chosen. Clears the histogram.
__global__ void __launch_bounds__(256) del_select_pick_k(DelSelect* st, uint32_t* hist,
                                                         int shift) {
  __shared__ int64_t c[256];
  const int d = threadIdx.x;
  const int64_t h = hist[d];
  c[d] = h;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {             // inclusive scan (Hillis-Steele)
    const int64_t v = d >= o ? c[d - o] : 0;
    __syncthreads();
    c[d] += v;
    __syncthreads();
  }
  const int64_t before = c[d] - h;
  const int64_t want = st->want;
  __syncthreads();
  if (h > 0 && before < want && want <= c[d]) {
    st->prefix |= (uint64_t)d << shift;
    st->mask |= (uint64_t)255 << shift;
    st->want = want - before;
  }
  hist[d] = 0;
}

// Keys equal to the threshold (in index order, so ties go as a stable sort would).
struct DelTie {
  const DelSelect* st;
  __device__ int32_t operator()(uint64_t k, int64_t) const { return k == st->prefix ? 1 : 0; }
};

// Below the threshold key, or among its first `want` ties (tie_pos: exclusive scan of
// the ties), a synapse goes.
__global__ void __launch_bounds__(kPlastBlock) del_select_mark_k(
    const uint64_t* __restrict__ key, DevCount m, const DelSelect* st,
    const int32_t* __restrict__ tie_pos, SynList L, int64_t n, uint8_t* __restrict__ dead,
    int32_t* bound) {
  const int64_t want = st->want;
  if (want <= 0) return;
  const int64_t m_ = m.get();
  const uint64_t kt = st->prefix;
  for (int64_t s = gtid(); s < m_; s += gstride()) {
    const uint64_t k = key[s];
    if (k < kt || (k == kt && tie_pos[s] < want)) {
      dead[s] = 1;
      unbind(L, s, n, bound);
    }
  }
}

__global__ void __launch_bounds__(kPlastBlock) excess_k(const int32_t* __restrict__ bound_k,
                                                       const double* __restrict__ z_k, int64_t n,
                                                       int32_t* __restrict__ exc) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  exc[j] = bound_k[j] - (int32_t)floor(z_k[j]);
}

// Owner of synapse s for element kind k, or -1 if s binds no element of that kind.
__device__ __forceinline__ int32_t owner_of(const SynList& L, int64_t s, int k) {
  if (k == 0) return L.src[s];
  return (int)L.type[s] == k - 1 ? L.tgt[s] : -1;
}

struct RetractFlag {            // live synapse of a neuron with an excess of kind k
  SynList L;
  const uint8_t* dead;
  const int32_t* exc;
  int k;
  __device__ int32_t operator()(int32_t, int64_t s) const {
    if (dead[s]) return 0;
    const int32_t o = owner_of(L, s, k);
    return (o >= 0 && exc[o] > 0) ? 1 : 0;
  }
};

// The candidate flags of one kind, once (the scan and the key pass read the bytes).
__global__ void __launch_bounds__(kPlastBlock) retract_flag_k(RetractFlag F, DevCount m,
                                                             uint8_t* __restrict__ flag) {
  const int64_t m_ = m.get();
  for (int64_t s = gtid(); s < m_; s += gstride()) flag[s] = (uint8_t)F(0, s);
}

struct ByteCount {
  __device__ int32_t operator()(uint8_t a, int64_t) const { return (int32_t)a; }
};

__global__ void __launch_bounds__(kPlastBlock) cand_write_k(RetractFlag F, const int32_t* __restrict__ pos,
                                                           DevCount m, uint64_t seed, DevStep step,
                                                           uint64_t* __restrict__ key,
                                                           int32_t* __restrict__ val) {
  const int64_t m_ = m.get();
  const uint64_t st = step.get();
  for (int64_t s = gtid(); s < m_; s += gstride()) {
    if (pos[s + 1] == pos[s]) continue;       // not a candidate (pos: the flags' scan)
    const int32_t o = owner_of(F.L, s, F.k);
    const uint64_t q = philox_word0(seed, 4, (uint64_t)s, st, (uint64_t)F.k, 0) >> 32;
    key[pos[s]] = ((uint64_t)(uint32_t)o << 32) | q;
    val[pos[s]] = (int32_t)s;
  }
}

// Candidates sorted by (owner, priority, s): the first exc[owner] of each owner go.
__global__ void __launch_bounds__(kPlastBlock) retract_k(const uint64_t* __restrict__ key,
                                                        const int32_t* __restrict__ val,
                                                        DevCount cnt, const int32_t* __restrict__ exc,
                                                        SynList L, int64_t n,
                                                        uint8_t* __restrict__ dead, int32_t* bound) {
  const int64_t c = cnt.get();
  for (int64_t p = gtid(); p < c; p += gstride()) {
    const uint64_t o = key[p] >> 32;
    // first candidate of this owner
    int64_t lo = 0, hi = p;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((key[mid] >> 32) < o) lo = mid + 1; else hi = mid;
    }
    if (p - lo < (int64_t)exc[o]) {
      const int64_t s = val[p];
      dead[s] = 1;
      unbind(L, s, n, bound);
    }
  }
}

struct LiveFlag {
  const uint8_t* dead;
  __device__ int32_t operator()(int32_t, int64_t s) const { return dead[s] ? 0 : 1; }
};

__global__ void __launch_bounds__(kPlastBlock) compact_k(SynList in, const uint8_t* __restrict__ dead,
                                                        const int32_t* __restrict__ pos, DevCount m,
                                                        SynList out) {
  const int64_t m_ = m.get();
  for (int64_t s = gtid(); s < m_; s += gstride()) {
    if (dead[s]) continue;
    const int64_t p = pos[s];
    out.src[p] = in.src[s];
    out.tgt[p] = in.tgt[s];
    out.type[p] = in.type[s];
  }
}

// The first `cnt` synapses of one list into another.
__global__ void __launch_bounds__(kPlastBlock) copy_list_k(SynList from, DevCount cnt, SynList to) {
  const int64_t c = cnt.get();
  for (int64_t s = gtid(); s < c; s += gstride()) {
    to.src[s] = from.src[s];
    to.tgt[s] = from.tgt[s];
    to.type[s] = from.type[s];
  }
}

// A count the device found (a scan total at position *at of `pos`) as a 64-bit and a
// 32-bit scalar.
__global__ void take_count_k(const int32_t* __restrict__ pos, DevCount at, int64_t* c64,
                             int32_t* c32) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int32_t c = pos[at.get()];
  if (c64) *c64 = c;
  if (c32) *c32 = c;
}

__global__ void __launch_bounds__(kPlastBlock) vacancy_k(const double* __restrict__ z,
                                                        const int32_t* __restrict__ bound,
                                                        int64_t n, int32_t* va, int32_t* ve,
                                                        int32_t* vi) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 3 * n) return;
  const int64_t k = g / n, j = g - k * n;
  int32_t* out = k == 0 ? va : k == 1 ? ve : vi;
  out[j] = (int32_t)floor(z[g]) - bound[g];
}

// New synapses (appended by the caller) bind their elements.
__global__ void __launch_bounds__(kPlastBlock) bind_k(const int32_t* __restrict__ src,
                                                     const int32_t* __restrict__ tgt,
                                                     const uint8_t* __restrict__ type,
                                                     DevCount cnt, int64_t n, int32_t* bound,
                                                     int32_t* err) {
  const int64_t c = cnt.get();
  for (int64_t q = gtid(); q < c; q += gstride()) {
    const int32_t i = src[q], g = tgt[q];
    const uint8_t ty = type[q];
    if (i < 0 || i >= n || g < 0 || g >= n || ty > 1) {
      atomicOr(err, 1);
      continue;
    }
    atomicAdd(&bound[i], 1);
    atomicAdd(&bound[(1 + (int64_t)ty) * n + g], 1);
  }
}

// Appends the *cnt synapses of `from` to the list L after its *m entries and binds
// their elements, if the list (capacity cap) holds them all; else appends nothing and
// sets kRecordCapacity in *flags. record_end_k then advances *m.
constexpr int32_t kRecordCapacity = 1;

__global__ void __launch_bounds__(kPlastBlock) record_k(SynList from, DevCount cnt, SynList L,
                                                       const int64_t* __restrict__ m, int64_t cap,
                                                       int64_t n, int32_t* bound, int32_t* flags) {
  const int64_t c = cnt.get();
  const int64_t base = *m;
  if (c == 0) return;
  if (base + c > cap) {
    if (gtid() == 0) atomicOr(flags, kRecordCapacity);
    return;
  }
  for (int64_t q = gtid(); q < c; q += gstride()) {
    const int32_t i = from.src[q], g = from.tgt[q];
    const uint8_t ty = from.type[q];
    L.src[base + q] = i;
    L.tgt[base + q] = g;
    L.type[base + q] = ty;
    atomicAdd(&bound[i], 1);
    atomicAdd(&bound[(1 + (int64_t)ty) * n + g], 1);
  }
}

__global__ void record_end_k(DevCount cnt, int64_t* m, int64_t cap) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t c = cnt.get();
  if (*m + c <= cap) *m += c;
}

__global__ void __launch_bounds__(kPlastBlock) fill_u8_k(uint8_t* p, DevCount n, uint8_t v) {
  const int64_t c = n.get();
  for (int64_t i = gtid(); i < c; i += gstride()) p[i] = v;
}

}  // namespace msp
