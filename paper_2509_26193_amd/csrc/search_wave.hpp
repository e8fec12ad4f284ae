// Wave-coherent Barnes-Hut search, in two kernels.
//
// search_sweep_k: the 64 lanes of a wavefront hold 64 sources adjacent in Morton
// order (and of one type) and walk the union of their level-0 expansions together.
// The node at the wave's position is read once (uniform address: scalar loads) and
// every lane applies its own rules to it:
//   - a lane is active at node x unless x lies inside a subtree it has already
//     accepted or skipped (x < mask_end), so each lane sees exactly the nodes of its
//     own depth-first walk, in the same order;
//   - the wave descends into x if any active lane opens it, otherwise jumps over
//     the subtree.
// It produces each source's level-0 normaliser Z and, every `interval` wave steps,
// a checkpoint per lane (running sum, mask_end) with the wave position.
//
// Parts: where a simulation has few tiles, each tile's pre-order range is cut into
// 2^p consecutive parts walked by different waves (a work unit is a tile's part).
// A part's walk starts from the lane states at its first node, found from that node's
// ancestors, so every lane sees the same nodes as in one walk; the part sums add up
// to Z and every part keeps its own checkpoints (running sums from the part's start).
//
// search_draw_k: one thread per source and element j: T = u Z, then the source's
// own walk restarts from the last checkpoint whose running sum does not exceed T
// (not from the root), then restart levels (a drawn cell) run per thread.
#pragma once

#include "search.hpp"

namespace msp {

constexpr int kCkptMax = 256;      // checkpoint slots per tile: this many where memory
constexpr int kCkptMin = 32;       // allows, else this many (both powers of two)
constexpr int kCkptStepMin = 16;   // smallest checkpoint interval, wave steps
constexpr int kPartLogMax = 3;     // at most 2^3 parts per tile
constexpr int kPartUnits = 131072; // parts are added while a simulation's units stay
                                   // within this (16 per wave of a full launch)
constexpr int kWaveBlock = 256;    // 4 independent waves per block
constexpr int kXcd = 8;            // accelerator dies; workgroup b runs on die b % 8
constexpr uint32_t kAheadBytes = 256;   // the sweep requests the records this far ahead
                                        // of its position into the L2
constexpr int64_t kAheadRecords = kAheadBytes / sizeof(NodeRec);   // room kept after the
                                        // sentinel record for those requests
constexpr int kRawBufferWord3 = 0x00020000;   // buffer descriptor word 3: raw dwords

// Requests of the second phase of a two-phase search (one simulation): one entry per
// element e; key[e] is the deferred cell's pre-order index >> shift, or `none` if the
// element was finished in the first phase. Sorting by key groups the requests by
// pre-order range, and the pre-order makes every subtree (a branch cell's in
// particular) one contiguous range.
struct DeferOut {
  int depth = kNoDefer;            // cells at this depth or deeper are deferred
  int shift = 0;
  uint64_t none = ~0ull;
  uint64_t* key = nullptr;         // [S]
  int32_t* val = nullptr;          // [S] e
  int32_t* cell = nullptr;         // [S] the deferred cell
  int32_t* src = nullptr;          // [S] source neuron
  int32_t* elem = nullptr;         // [S] element j of the source
  uint8_t* level = nullptr;        // [S] level of the deferred expansion
};

struct SweepOut {
  double* Z;                       // [units][64] level-0 sum of the unit's part
  int32_t* v0;                     // [units][64] level-0 visits (counting launches only)
  int32_t* o0;                     // [units][64] level-0 opens
  int32_t* e0;                     // [units][64] level-0 accepted entries
  int32_t* nck;                    // [units] checkpoints written
  int32_t* ck_x;                   // [ck_units][ck_slots] wave position
  double* ck_P;                    // [ck_units][ck_slots][64] running sum
  int32_t* ck_me;                  // [ck_units][ck_slots][64] mask_end
  int ck_slots;                    // checkpoint slots per region: kCkptMax or kCkptMin
  int64_t ck_units;                // checkpoint regions (see unit_slots)
  const int32_t* tile_count;       // device scalar
  const int32_t* unit_count;       // device scalar: tiles times their parts
  int32_t* queue;                  // [kXcd] tile counters, zero at launch
  unsigned long long* wave_steps;  // counting launches: total wave steps (nullable)
  DeferOut defer;                  // two-phase search (depth kNoDefer: one phase)
};

// Read-only data seen through the constant address space: wave-uniform loads from
// it become scalar loads into SGPRs (the data is not written during the search).
template <class T>
using cptr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
}

// Record x as one 32-byte scalar load with a 32-bit byte offset in a register (no
// per-node 64-bit address arithmetic; the empty asm keeps the compiler from widening
// the offset computation to 64 bits).
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ NodeRec load_rec_u(cptr<NodeRec> R, uint32_t x) {
  uint32_t off = x * (uint32_t)sizeof(NodeRec);
  asm("" : "+s"(off));
  const u32x8 w =
      *(cptr<u32x8>)((const __attribute__((address_space(4))) char*)R + off);
  NodeRec r;
  r.x = __builtin_bit_cast(double, ((uint64_t)w[1] << 32) | w[0]);
  r.y = __builtin_bit_cast(double, ((uint64_t)w[3] << 32) | w[2]);
  r.z = __builtin_bit_cast(double, ((uint64_t)w[5] << 32) | w[4]);
  r.v = (int32_t)w[6];
  r.meta = w[7];
  return r;
}

// Record at byte offset `off` (a multiple of the record size).
__device__ __forceinline__ NodeRec load_rec_b(cptr<NodeRec> R, uint32_t off) {
  const u32x8 w =
      *(cptr<u32x8>)((const __attribute__((address_space(4))) char*)R + off);
  NodeRec r;
  r.x = __builtin_bit_cast(double, ((uint64_t)w[1] << 32) | w[0]);
  r.y = __builtin_bit_cast(double, ((uint64_t)w[3] << 32) | w[2]);
  r.z = __builtin_bit_cast(double, ((uint64_t)w[5] << 32) | w[4]);
  r.v = (int32_t)w[6];
  r.meta = w[7];
  return r;
}

__device__ __forceinline__ NodeRec load_rec(cptr<NodeRec> R, int64_t x) {
  NodeRec r;
  r.x = R[x].x;
  r.y = R[x].y;
  r.z = R[x].z;
  r.v = R[x].v;
  r.meta = R[x].meta;
  return r;
}

// The pre-order range [x_lo, x_hi) of part `part` of a tile cut into 2^plog parts
// (wave-uniform; every wave that walks a part of the tile finds the same cuts). The
// cuts lie around m, the median of the sources' leaf positions, at m - c s and m + c s
// for a ladder of multipliers c (8 parts: 1, 8, 64; 4 parts: 4; 2 parts: m alone), s
// being the sources' leaf range (at least 64), clamped into [1, end]: the union walk's
// steps are densest around the sources and thin out with the distance from them along
// the pre-order.
__device__ __forceinline__ void part_range(int32_t li, bool valid, int lane, int plog, int part,
                                           int32_t end, int32_t& x_lo, int32_t& x_hi) {
  const int32_t key = valid ? li : INT32_MAX;
  int32_t lo = INT32_MAX, hi = -1, rank = 0;
  for (int m = 0; m < kWave; ++m) {
    const int32_t km = __builtin_amdgcn_readlane(key, m);
    if (km != INT32_MAX) {
      lo = km < lo ? km : lo;
      hi = km > hi ? km : hi;
    }
    rank += (km < key || (km == key && m < lane)) ? 1 : 0;
  }
  const int nv = __popcll(__ballot(valid));
  const uint64_t at = __ballot(valid && rank == nv / 2);
  const int32_t med = __builtin_amdgcn_readlane(key, __ffsll((unsigned long long)at) - 1);
  const int64_t span = (int64_t)hi - lo + 1 > 64 ? (int64_t)hi - lo + 1 : 64;
  const int np = 1 << plog;
  // cut k (1 <= k < np) at med + mult(k - np / 2) span
  auto cut = [&](int k) -> int32_t {
    const int c = k - np / 2;
    const int a = c < 0 ? -c : c;
    int64_t mult = 0;
    if (a != 0) mult = plog == 3 ? (a == 1 ? 1 : a == 2 ? 8 : 64) : 4;
    int64_t x = (int64_t)med + (c < 0 ? -mult : mult) * span;
    x = x < 1 ? 1 : x;
    return (int32_t)(x > end ? end : x);
  };
  x_lo = __builtin_amdgcn_readfirstlane(part == 0 ? 1 : cut(part));
  x_hi = __builtin_amdgcn_readfirstlane(part == np - 1 ? end : cut(part + 1));
}

// The checkpoint slots of unit `unit`, part `part` of its tile's 2^plog parts: the
// first slot and the count. Where the launch has no more units than checkpoint
// regions (W.ck_units, one per tile of the largest launch), every unit has a region
// of its own; otherwise the parts of a tile share its region equally.
__device__ __forceinline__ void unit_slots(int slots, bool own, int64_t tile,
                                           int plog, int part, int64_t unit, int64_t& first,
                                           int& count) {
  if (own) {
    first = unit * slots;
    count = slots;
  } else {
    count = slots >> plog;
    first = tile * slots + (int64_t)part * count;
  }
}

// A lane's mask end at node x0 > 1 of a walk that starts there: the end of the
// subtree of the first ancestor of x0 that the lane's own walk does not enter
// (accepted, or holding no vacancy), else `me` unchanged (the lane is active at x0). The
// ancestors are found by following the pre-order from the root's first child:
// over a subtree that ends at or before x0, into one that holds it.
template <bool OWN>
__device__ __forceinline__ int32_t mask_at(const SearchArgs& A, cptr<NodeRec> R, int32_t x0,
                                           int32_t me, int32_t li, double xi, double yi,
                                           double zi) {
  int32_t y = 1;
  while (y < x0) {
    const NodeRec r = load_rec_u(R, (uint32_t)y);
    int32_t sk = y + 1;
    if ((int32_t)r.meta >= 0) {
      const int32_t e = (int32_t)(r.meta & kSkipMask);
      sk = e > y ? e : y + 1;
    }
    if (sk > x0) {                       // an ancestor of x0 (inner node)
      bool out = true;                   // v == 0: the walk jumps over the subtree
      if (r.v != 0) {
        const double d2 = dist2(xi, yi, zi, r.x, r.y, r.z);
        const bool contains = OWN && (uint32_t)(li - y) < (uint32_t)(sk - y);
        out = !contains && (OWN ? bh_accept_u(A.L2, A.theta2, d2, r.meta)
                                : bh_accept_d(A.acc_d2, d2, r.meta));
      }
      if (me <= y && out) me = sk;
      y = y + 1;
    } else {
      y = sk;
    }
  }
  return me;
}

// `step0`: initial checkpoint interval (a power of two), chosen from the length of
// the wave's previous sweep so that the buffer rarely has to be thinned out.
// Returns the number of wave steps of this unit: part `part` of the tile's 2^plog
// parts (unit index `unit`); own: the unit has a checkpoint region of its own.
// OWN: test whether an inner node holds the source's own leaf (such a node is always
// opened). Launches drop the test only where it can never fire: with theta <= 1/2 and
// every position inside the cube, the source and the node's centroid lie in (or,
// through rounding, within a tiny fraction of an edge of) the node's cell of edge l,
// so d^2 <= 3 l^2 (1 + 2^-4) and theta^2 d^2 < l^2: the acceptance test fails anyway.
template <bool DIAG, int SLOTS, bool OWN>
__device__ __forceinline__ int sweep_tile(const SearchArgs& A, const SweepOut& W, int tile,
                                          int part, int plog, int64_t unit, bool own, int lane,
                                          int step0) {
  const int64_t slot = (int64_t)tile * kWave + lane;
  const int32_t i = A.work[slot];                                // -1: padding lane
  const bool valid = i >= 0;
  const int32_t i0 = __builtin_amdgcn_readfirstlane(i);         // lane 0 is never padding
  const int t = A.type[i0] ? 1 : 0;
  const cptr<NodeRec> R = as_const(A.rec[t]);
  int32_t li = -1;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (valid) {
    li = A.leaf_of[i];
    xi = A.pos[3 * (int64_t)i];
    yi = A.pos[3 * (int64_t)i + 1];
    zi = A.pos[3 * (int64_t)i + 2];
  }
  // complete the source loads before the walk: inside it, checkpoint stores share
  // the vector-memory counter and would otherwise make every use of the source
  // coordinates wait for them
  __builtin_amdgcn_s_waitcnt(0x0F70);      // vmcnt(0)
  SumPass sum{A.k2};
  Count c0;
  int nck = 0;
  int steps = 0;
  const NodeRec root = load_rec(R, 0);
  if (root.meta & kLeafBit) {
    // a one-neuron tree: the only neuron is the source itself, so the list is empty
    if (DIAG && valid && part == 0) c0.visits = 1;
  } else {
    const int32_t root_end = (int32_t)(root.meta & kSkipMask);
    int32_t x = 1, end = root_end;
    int32_t me = valid ? 0 : 0x7FFFFFFF;     // padding lanes are never active
    if (plog > 0) {
      part_range(li, valid, lane, plog, part, root_end, x, end);
      if (x > 1 && x < end) me = mask_at<OWN>(A, R, x, me, li, xi, yi, zi);
    }
    int64_t ck0 = 0;                        // this unit's checkpoint slots
    int ns = 0;
    unit_slots(SLOTS, own, tile, plog, part, unit, ck0, ns);
    int32_t* ckx = W.ck_x + ck0;
    double* ckP = W.ck_P + ck0 * kWave + lane;
    int32_t* ckme = W.ck_me + ck0 * kWave + lane;
    if (DIAG && valid && part == 0) {
      c0.visits = 1;
      c0.opens = 1;
    }
    // Steps are counted in `ph`: the step index modulo the checkpoint interval (a power
    // of two, 2^32 / inc), kept in the top bits, so that it is 0 exactly at the
    // multiples of the interval and the step needs no separate test; s1 is the next
    // multiple to be reached (the current one while ph is 0).
    uint32_t inc = 1u << (32 - __builtin_ctz((uint32_t)__builtin_amdgcn_readfirstlane(step0)));
    uint32_t ph = 0;
    int s1 = 0;
    // the walk counts positions in bytes of the record array (position x at 32 x):
    // the next record's address is then the position itself
    constexpr int kRecShift = 5;
    static_assert(sizeof(NodeRec) == (1 << kRecShift), "32-byte records");
    // (unsigned: up to kMaxNodes positions, the sentinel's offset is 2^31)
    uint32_t xb = (uint32_t)x << kRecShift;
    const uint32_t endb = (uint32_t)end << kRecShift;
    uint32_t meb = valid ? (uint32_t)me << kRecShift : ~0u;  // padding lanes: never active
    const uint32_t lib = (uint32_t)li << kRecShift;
    NodeRec cur = load_rec_b(R, xb);
    // Most wave steps go to a record a little ahead of the current one (the next one,
    // or the end of a small subtree), and a record that misses the L2 costs the step a
    // trip to the Infinity Cache or HBM. Every step therefore also requests the line
    // kAheadBytes past the new position into the L2: a buffer load whose data goes to
    // local memory (one scratch word per lane, never read), so that it holds no register
    // and nothing ever waits for it. The record array keeps kAheadRecords of room after
    // the sentinel (the position is at most the sentinel's), and the buffer covers them.
    // The distance is the instruction's immediate offset, which the hardware may also add
    // to the local-memory address: the sink keeps that much room after the last wave's
    // words, so every write stays inside the block's own local memory either way.
    __shared__ uint32_t ahead_sink[kWaveBlock + kAheadBytes / sizeof(uint32_t)];
    const __amdgpu_buffer_rsrc_t ahead_buf = __builtin_amdgcn_make_buffer_rsrc(
        (void*)R, (short)0, (int)((uint32_t)(root_end + 1 + kAheadRecords) << kRecShift),
        kRawBufferWord3);
    auto* ahead_lds = (__attribute__((address_space(3))) void*)(
        ahead_sink + __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~(kWave - 1))));
    while (xb < endb) {
      if constexpr (SLOTS > 0) {
        // checkpoints at multiples of the interval; a full buffer keeps every other
        // one and doubles the interval
        if (ph == 0) {                    // step index s1
          bool store = true;
          if (nck == ns) {
#pragma unroll 1
            for (int k = 1; k < ns / 2; ++k) {
              ckP[k * kWave] = ckP[2 * k * kWave];
              ckme[k * kWave] = ckme[2 * k * kWave];
              if (lane == 0) ckx[k] = ckx[2 * k];
            }
            nck = ns / 2;
            inc >>= 1;
            const int half = (int)(1u << (31 - __builtin_ctz(inc)));   // the old interval
            if (s1 & half) {                // half way between multiples of the new one
              ph = 0x80000000u;
              s1 += half;
              store = false;
            }
          }
          if (store) {
            ckP[nck * kWave] = sum.Z;
            ckme[nck * kWave] = (int32_t)(meb >> kRecShift);
            if (lane == 0) ckx[nck] = (int32_t)(xb >> kRecShift);
            nck = __builtin_amdgcn_readfirstlane(nck + 1);
            s1 += (int)(1u << (32 - __builtin_ctz(inc)));   // the interval
          }
        }
      }
      // one node: uniform branches on its kind, per-lane decisions as lane masks, the
      // weight evaluated on every lane and added where the lane takes the entry. The
      // next record's load is issued as soon as the next node is known (a leaf's at
      // once, an inner node's after the ballot), so it is in flight while this node's
      // weights are computed.
      // Lane decisions are lane masks: a ballot of each compare (its mask itself),
      // combined on the scalar unit, and turned back into a lane condition where a
      // select needs one (inverse ballot: the same mask).
      const uint32_t meta = cur.meta;
      const uint64_t m_act = __builtin_amdgcn_ballot_w64(xb >= meb);
      const bool active = __builtin_amdgcn_inverse_ballot_w64(m_act);
      if (DIAG && active) c0.visits += 1;
      uint32_t next;                                         // bytes
      NodeRec nxt;
      if (__builtin_expect((int32_t)meta < 0, 0)) {          // leaf
        next = xb + (1 << kRecShift);                        // index N: the sentinel
        if (cur.v == 0) {
          nxt = load_rec_b(R, next);
        } else if (!(meta & kBucketBit)) {
          const int32_t id = (int32_t)(meta & kIdMask);
          const bool keep = active && id != i;
          if (DIAG && keep) c0.entries += 1;
          const double d2 = dist2(xi, yi, zi, cur.x, cur.y, cur.z);
          const double vd = (double)cur.v;
          // the record is no longer needed: its registers take the next one; the
          // weight is computed while the load is in flight (no instruction of it may
          // be scheduled above the load)
          nxt = load_rec_b(R, next);
          __builtin_amdgcn_sched_barrier(0);
          sum.Z = sum.Z + kernel_weight_vd(keep, vd, d2, A.k2);
        } else {                              // several neurons at one finest cell
          nxt = load_rec_b(R, next);
          const int32_t x = (int32_t)(xb >> kRecShift);
          const cptr<int32_t> vs = as_const(A.vs[t]);
          const cptr<int32_t> order = as_const(A.order);
          const cptr<double> pos = as_const(A.pos);
          const int32_t pe = as_const(A.nend)[x];
          for (int32_t p = as_const(A.nbeg)[x]; p < pe; ++p) {
            const int32_t id = order[p];
            const int32_t v = vs[p];
            if (v == 0) continue;
            if (DIAG && active && id != i) c0.entries += 1;
            sum.Z = sum.Z + kernel_weight_if(
                active && id != i, v,
                dist2(xi, yi, zi, pos[3 * (int64_t)id], pos[3 * (int64_t)id + 1],
                      pos[3 * (int64_t)id + 2]),
                A.k2);
          }
        }
      } else if (__builtin_expect(cur.v == 0, 0)) {   // no vacancy below: over the subtree
        next = (meta & kSkipMask) << kRecShift;
        nxt = load_rec_b(R, next);
      } else {                                               // inner node
        const uint32_t sk = (meta & kSkipMask) << kRecShift;   // > xb
        const double d2 = dist2(xi, yi, zi, cur.x, cur.y, cur.z);
        uint64_t m_far = __builtin_amdgcn_ballot_w64(
            OWN ? bh_accept_u(A.L2, A.theta2, d2, meta) : bh_accept_d(A.acc_d2, d2, meta));
        // li in [x, sk), as offsets (padding lanes have li = -1: far above, unsigned)
        if (OWN) m_far &= ~__builtin_amdgcn_ballot_w64(lib - xb < sk - xb);
        const uint64_t m_take = m_act & m_far;
        const bool take = __builtin_amdgcn_inverse_ballot_w64(m_take);
        const uint32_t me_next = take ? sk : meb; // (sk is then free for the next node)
        const double vd = (double)cur.v;
        // the wave descends iff a lane opens x; the record is no longer needed: its
        // registers take the next one. (The and-not sets the scalar condition code to
        // "some lane opens", which the select uses directly.)
        uint64_t m_open;
        asm("s_andn2_b64 %0, %2, %3\n\ts_cselect_b32 %1, %4, %5"
            : "=&s"(m_open), "=s"(next)
            : "s"(m_act), "s"(m_far), "s"(xb + (1 << kRecShift)), "s"(sk)
            : "scc");
        nxt = load_rec_b(R, next);
        __builtin_amdgcn_sched_barrier(0);
        sum.Z = sum.Z + kernel_weight_vd(take, vd, d2, A.k2);
        meb = me_next;
        if (DIAG && __builtin_amdgcn_inverse_ballot_w64(m_open)) c0.opens += 1;
        if (DIAG && take) c0.entries += 1;
      }
      xb = next;
      cur = nxt;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ahead_buf, ahead_lds, 4, 0, (int)xb,
                                               (int)kAheadBytes, 0);
      if (SLOTS > 0) {
        ph += inc;
      } else if (DIAG) {
        ++steps;
      }
    }
    if (SLOTS > 0) steps = s1 - (int)((0u - ph) >> __builtin_ctz(inc));
  }
  const int64_t us = unit * kWave + lane;
  if (lane == 0) W.nck[unit] = nck;
  W.Z[us] = sum.Z;
  if (DIAG) {
    W.v0[us] = c0.visits;
    W.o0[us] = c0.opens;
    W.e0[us] = c0.entries;
    if (W.wave_steps && lane == 0) atomicAdd(W.wave_steps, (unsigned long long)steps);
  }
  return steps;
}

// The draws and restarts of the source in worklist slot `slot` (DEFER: restarts from
// cells at depth >= W.defer.depth become second-phase requests). The slot's tile has
// 2^plog parts, units u0, u0 + 1, ... keep: the thread's memory for a restart level's
// entries (see restart_search).
template <bool DIAG, int SLOTS, bool DEFER>
__device__ __forceinline__ void draw_slot(const SearchArgs& A, const DiagOut& D, const SweepOut& W,
                                          int64_t slot, int64_t u0, int plog, bool own,
                                          const KeptEntries* keep) {
  const int32_t i = A.work[slot];
  if (i < 0) return;
  const int64_t tile = slot / kWave;
  const int lane = (int)(slot % kWave);
  const int t = A.type[i] ? 1 : 0;
  const NodeRec* __restrict__ R = A.rec[t];
  const int32_t* vs = A.vs[t];
  const int32_t li = A.leaf_of[i];
  const double xi = A.pos[3 * (int64_t)i], yi = A.pos[3 * (int64_t)i + 1],
               zi = A.pos[3 * (int64_t)i + 2];
  const int np = 1 << plog;
  const double* Zp = W.Z + u0 * kWave + lane;        // the part sums, in part order
  double Z = 0.0;
  for (int q = 0; q < np; ++q) Z = Z + Zp[q * kWave];
  const NodeRec root = R[0];             // Z > 0 implies an inner root
  const int32_t end = (int32_t)(root.meta & kSkipMask);
  const int32_t a = A.vac_axon[i];
  const int64_t off = A.elem_off[i];
  Count c0;
  if (DIAG) {
    for (int q = 0; q < np; ++q) {
      c0.visits += W.v0[(u0 + q) * kWave + lane];
      c0.opens += W.o0[(u0 + q) * kWave + lane];
      c0.entries += W.e0[(u0 + q) * kWave + lane];
    }
  }
  for (int32_t j = 0; j < a; ++j) {
    int lev = 1;
    Count c = c0;
    int32_t tgt = -1;
    int32_t deferred = -1;
    if (Z > 0.0) {
      const double T = draw_u(A.seed, i, j, A.step, 0) * Z;
      SelectPass p{A.k2, T};
      Count none;
      // the part where the running sum crosses T (the sums added as for Z), and T
      // from that part's start
      int k = -1;
      double Tk = T, pre = 0.0;
      for (int q = 0; q < np; ++q) {
        const double zq = Zp[q * kWave];
        const double nxt = pre + zq;
        if (k < 0 && zq > 0.0 && nxt > T) {
          k = q;
          Tk = T - pre;
        }
        pre = nxt;
      }
      if (k >= 0) {
        const int nck = W.nck[u0 + k];
        int64_t ck0 = 0;
        int ns = 0;
        unit_slots(SLOTS, own, tile, plog, k, u0 + k, ck0, ns);
        const int32_t* ckx = W.ck_x + ck0;
        const double* ckP = W.ck_P + ck0 * kWave + lane;
        const int32_t* ckme = W.ck_me + ck0 * kWave + lane;
        // last checkpoint whose running sum does not exceed Tk (checkpoint 0 holds 0)
        int lo = 0, hi = nck - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (ckP[mid * kWave] <= Tk) lo = mid; else hi = mid - 1;
        }
        p.P = ckP[lo * kWave];
        p.T = Tk;
        const int32_t cx = ckx[lo], cm = ckme[lo * kWave];
        expand_range<false>(A, R, vs, cx > cm ? cx : cm, end, i, li, xi, yi, zi, p, none);
      }
      if (p.chosen < 0) {                       // not crossed (rounding): full walk
        p = SelectPass{A.k2, T};
        expand_range<false>(A, R, vs, 1, end, i, li, xi, yi, zi, p, none);
      }
      const int32_t id = p.chosen >= 0 ? p.chosen : p.last;
      const bool neuron = p.chosen >= 0 ? p.chosen_neuron : p.last_neuron;
      if (id >= 0)
        tgt = neuron ? id
                     : restart_search<DIAG, DEFER>(A, R, vs, id, 1, W.defer.depth, i, j, li,
                                                   xi, yi, zi, &lev, c, &deferred, keep);
    }
    if (DEFER) {
      const int64_t e = off + j;
      if (tgt == kDeferred) {
        W.defer.key[e] = (uint64_t)((uint32_t)deferred >> W.defer.shift);
        W.defer.cell[e] = deferred;
        W.defer.src[e] = i;
        W.defer.elem[e] = j;
        W.defer.level[e] = (uint8_t)lev;
        tgt = -1;                               // the second phase overwrites it
      } else {
        W.defer.key[e] = W.defer.none;
      }
      W.defer.val[e] = (int32_t)e;
    }
    A.target[off + j] = tgt;
    if (DIAG) {
      if (D.z0) D.z0[off + j] = Z;
      if (D.levels) D.levels[off + j] = lev;
      if (D.visits) D.visits[off + j] = c.visits;
      if (D.opens) D.opens[off + j] = c.opens;
      if (D.visits0) D.visits0[off + j] = c0.visits;
      if (D.opens0) D.opens0[off + j] = c0.opens;
      if (D.entries0) D.entries0[off + j] = c0.entries;
    }
  }
}

}  // namespace msp
