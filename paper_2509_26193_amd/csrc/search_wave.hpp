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
// It produces each source's level-0 normaliser (sum and shift) and, every
// `interval` wave steps, a checkpoint per lane (running sum, shift, mask_end) with
// the wave position.
//
// search_draw_k: one thread per source and element j: T = u Z, then the source's
// own walk restarts from the last checkpoint whose running sum does not exceed T
// (not from the root), then restart levels (a drawn cell) run per thread.
#pragma once

#include "search.hpp"

namespace msp {

constexpr int kCkpt = 32;          // checkpoint slots per tile
constexpr int kCkptStep0 = 32;     // initial checkpoint interval, wave steps
constexpr int kWaveBlock = 256;    // 4 independent waves per block
constexpr int kXcd = 8;            // accelerator dies; workgroup b runs on die b % 8
constexpr int32_t kNoShift = 0x7FFFFFFF;

struct SweepOut {
  double* Z;                       // [slots] level-0 sum at shift s
  int32_t* s;                      // [slots]
  int32_t* v0;                     // [slots] level-0 visits (counting launches only)
  int32_t* o0;                     // [slots] level-0 opens
  int32_t* nck;                    // [tiles] checkpoints written
  int32_t* ck_x;                   // [tiles][kCkpt] wave position
  double* ck_P;                    // [tiles][kCkpt][64] running sum
  int32_t* ck_s;                   // [tiles][kCkpt][64] shift of the running sum
  int32_t* ck_me;                  // [tiles][kCkpt][64] mask_end
  const int32_t* tile_count;       // device scalar
  int32_t* queue;                  // [kXcd] tile counters, zero at launch
};

// Read-only data seen through the constant address space: wave-uniform loads from
// it become scalar loads into SGPRs (the data is not written during the search).
template <class T>
using cptr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
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

template <bool DIAG>
__device__ __forceinline__ void sweep_tile(const SearchArgs& A, const SweepOut& W, int tile,
                                           int lane) {
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
  SumPass sum{A.inv_s2};
  Count c0;
  int nck = 0;
  const NodeRec root = load_rec(R, 0);
  if (root.meta & kLeafBit) {
    // a one-neuron tree: the only neuron is the source itself, so the list is empty
    if (DIAG && valid) c0.visits = 1;
  } else {
    const int32_t end = (int32_t)(root.meta & kSkipMask);
    int32_t* ckx = W.ck_x + (int64_t)tile * kCkpt;
    double* ckP = W.ck_P + (int64_t)tile * kCkpt * kWave + lane;
    int32_t* cks = W.ck_s + (int64_t)tile * kCkpt * kWave + lane;
    int32_t* ckme = W.ck_me + (int64_t)tile * kCkpt * kWave + lane;
    if (DIAG && valid) {
      c0.visits = 1;
      c0.opens = 1;
    }
    int32_t x = 1;
    int32_t me = valid ? 0 : 0x7FFFFFFF;     // padding lanes are never active
    int steps = 0, imask = kCkptStep0 - 1;   // checkpoint interval - 1 (a power of 2)
    while (x < end) {
      if ((steps & imask) == 0) {
        if (nck == kCkpt) {                   // full: keep every other checkpoint
#pragma unroll 1
          for (int k = 1; k < kCkpt / 2; ++k) {
            ckP[k * kWave] = ckP[2 * k * kWave];
            cks[k * kWave] = cks[2 * k * kWave];
            ckme[k * kWave] = ckme[2 * k * kWave];
            if (lane == 0) ckx[k] = ckx[2 * k];
          }
          nck = kCkpt / 2;
          imask = 2 * imask + 1;
        }
        if ((steps & imask) == 0) {
          ckP[nck * kWave] = sum.Z;
          cks[nck * kWave] = sum.s;
          ckme[nck * kWave] = me;
          if (lane == 0) ckx[nck] = x;
          ++nck;
        }
      }
      ++steps;
      const NodeRec cur = load_rec(R, x);
      const bool active = x >= me;
      if (DIAG && active) c0.visits += 1;
      const uint32_t meta = cur.meta;
      if (meta & kLeafBit) {
        if (cur.v != 0) {
          if (!(meta & kBucketBit)) {
            const int32_t id = (int32_t)(meta & kIdMask);
            if (active && id != i) sum(id, true, cur.v, dist2(xi, yi, zi, cur.x, cur.y, cur.z));
          } else {
            const cptr<int32_t> vs = as_const(A.vs[t]);
            const cptr<int32_t> order = as_const(A.order);
            const cptr<double> pos = as_const(A.pos);
            const int32_t pe = as_const(A.nend)[x];
            for (int32_t p = as_const(A.nbeg)[x]; p < pe; ++p) {
              const int32_t id = order[p];
              const int32_t v = vs[p];
              if (active && id != i && v != 0)
                sum(id, true, v, dist2(xi, yi, zi, pos[3 * (int64_t)id], pos[3 * (int64_t)id + 1],
                                       pos[3 * (int64_t)id + 2]));
            }
          }
        }
        x = x + 1;
        continue;
      }
      int32_t sk = (int32_t)(meta & kSkipMask);
      sk = sk > x ? sk : x + 1;
      if (cur.v == 0) {
        x = sk;
        continue;
      }
      const bool contains = li >= x && li < sk;
      const double d2 = dist2(xi, yi, zi, cur.x, cur.y, cur.z);
      const int dep = (int)((meta >> kSkipBits) & 31u);
      const bool acc_ok = ldexp(A.L2, -2 * dep) < A.theta2 * d2;
      const bool open = active && (contains || !acc_ok);
      if (active && !contains && acc_ok) {
        sum(x, false, cur.v, d2);
        me = sk;
      }
      if (DIAG && open) c0.opens += 1;
      x = __any(open) ? x + 1 : sk;
    }
  }
  if (lane == 0) W.nck[tile] = nck;
  W.Z[slot] = sum.Z;
  W.s[slot] = sum.s;
  if (DIAG) {
    W.v0[slot] = c0.visits;
    W.o0[slot] = c0.opens;
  }
}

// Persistent waves pull 64-source tiles: first from the Morton range of their own
// die (neighbouring sources share upper-tree nodes in that die's L2), then from the
// other dies' ranges.
template <bool DIAG>
__global__ void __launch_bounds__(kWaveBlock) search_sweep_k(SearchArgs A, SweepOut W) {
  const int lane = threadIdx.x & (kWave - 1);
  const int home = blockIdx.x % kXcd;
  const int ntiles = *W.tile_count;
  int q = 0;
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
    sweep_tile<DIAG>(A, W, lo + got, lane);
  }
}

// One thread per worklist slot (source): its elements' draws and restarts.
template <bool DIAG>
__global__ void __launch_bounds__(256) search_draw_k(SearchArgs A, DiagOut D, SweepOut W) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= (int64_t)(*W.tile_count) * kWave) return;
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
  const double Z = W.Z[slot];
  const int32_t s = W.s[slot];
  const int nck = W.nck[tile];
  const NodeRec root = R[0];             // Z > 0 implies an inner root
  const int32_t end = (int32_t)(root.meta & kSkipMask);
  const int32_t* ckx = W.ck_x + tile * kCkpt;
  const double* ckP = W.ck_P + tile * kCkpt * kWave + lane;
  const int32_t* cks = W.ck_s + tile * kCkpt * kWave + lane;
  const int32_t* ckme = W.ck_me + tile * kCkpt * kWave + lane;
  const int32_t a = A.vac_axon[i];
  const int64_t off = A.elem_off[i];
  const double z0 = Z > 0.0 ? ldexp(Z, -s) : 0.0;
  Count c0;
  if (DIAG) {
    c0.visits = W.v0[slot];
    c0.opens = W.o0[slot];
  }
  for (int32_t j = 0; j < a; ++j) {
    int lev = 1;
    Count c = c0;
    int32_t tgt = -1;
    if (Z > 0.0) {
      const double T = draw_u(A.seed, i, j, A.step, 0) * Z;
      SelectPass p{A.inv_s2, s, T};
      Count none;
      {
        // last checkpoint whose running sum (at the final shift) does not exceed T
        int lo = 0, hi = nck - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          const int32_t sm = cks[mid * kWave];
          const double pm = sm == kNoShift ? 0.0 : ldexp(ckP[mid * kWave], s - sm);
          if (pm <= T) lo = mid; else hi = mid - 1;
        }
        const int32_t sl = cks[lo * kWave];
        p.P = sl == kNoShift ? 0.0 : ldexp(ckP[lo * kWave], s - sl);
        const int32_t cx = ckx[lo], cm = ckme[lo * kWave];
        expand_range<false>(A, R, vs, cx > cm ? cx : cm, end, i, li, xi, yi, zi, p, none);
        if (p.chosen < 0) {                       // not crossed (rounding): full walk
          p = SelectPass{A.inv_s2, s, T};
          expand_range<false>(A, R, vs, 1, end, i, li, xi, yi, zi, p, none);
        }
      }
      const int32_t id = p.chosen >= 0 ? p.chosen : p.last;
      const bool neuron = p.chosen >= 0 ? p.chosen_neuron : p.last_neuron;
      if (id >= 0)
        tgt = neuron ? id : restart_search<DIAG>(A, R, vs, id, i, j, li, xi, yi, zi, &lev, c);
    }
    A.target[off + j] = tgt;
    if (DIAG) {
      if (D.z0) D.z0[off + j] = z0;
      if (D.levels) D.levels[off + j] = lev;
      if (D.visits) D.visits[off + j] = c.visits;
      if (D.opens) D.opens[off + j] = c.opens;
      if (D.visits0) D.visits0[off + j] = c0.visits;
      if (D.opens0) D.opens0[off + j] = c0.opens;
    }
  }
}

}  // namespace msp
