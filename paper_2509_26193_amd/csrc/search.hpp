// Barnes-Hut target search (Sec. III-B, "Division of work"; Sec. III-A, "Update of
// synapses"). For every vacant axonal element of source i (type t):
//   * expand a start cell S (first the root): walk its subtree in depth-first
//     pre-order; a node with no type-t vacancy is skipped, a leaf (a neuron other
//     than i) is always accepted, a cell containing i is opened, any other cell is
//     accepted iff l^2 < theta^2 d^2 (l = edge, d = distance from i to the cell's
//     type-t centroid) and opened otherwise;
//   * weight each accepted entry by v * exp(-d^2 / sigma^2), draw u from Philox and
//     take the first entry whose running sum exceeds u * Z;
//   * a neuron ends the search; a cell becomes the next start cell (restart).
// Acceptance decisions are evaluated in float64 exactly as written (no contraction),
// weight mantissas in float32, weights and running sums in float64.
#pragma once

#include <float.h>
#include <math.h>

#include "common.hpp"

namespace msp {

constexpr double kLog2e = 1.4426950408889634074;
// exp(-x) is 0 in float64 beyond this x; such entries carry no weight.
constexpr double kUnderflowX = 745.13321910194110842;
constexpr int kMaxLevels = 64;

struct SearchArgs {
  const NodeRec* rec[2];
  const int32_t* vs[2];          // per-type counts in sorted order (bucket members)
  const double* pos;
  const int32_t* order;
  const int32_t* nbeg;
  const int32_t* nend;
  const int32_t* leaf_of;
  bool own;                      // test for the source's own cell (see own_cell_needed)
  const uint8_t* type;
  const int32_t* vac_axon;
  const int64_t* elem_off;
  const int32_t* work;           // sources with a_i > 0, in search order (-1: padding)
  int32_t* target;
  int32_t* err;
  double L2;                     // box_edge * box_edge
  double theta2;                 // theta * theta
  double acc_d2;                 // accept_bound(L2, theta2) (walks without the own-cell test)
  double k2;                     // log2(e) / (sigma * sigma)
  uint64_t seed, step;
};

// Kernel weight v * exp(-x), x = d^2 / sigma^2, built in float64 from y = x log2(e):
// y = fl + fr (fl integer, 0 <= fr < 1), weight = ldexp(v * 2^-fr, -fl), with the
// mantissa 2^-fr from the float32 hardware exp2 (fr is in [0, 1), so 2^-fr is a
// normal float in (1/2, 1] and needs no range reduction). The float64 exponent range
// holds every weight the float64 definition does not flush to zero, so running sums
// need no rescaling and the sum and selection passes add identical terms in the same
// order (bitwise equal prefix sums).
constexpr double kMaxY = kUnderflowX * kLog2e;   // exp(-x) == 0 in float64 beyond this

// Barnes-Hut acceptance of an inner node at depth dep (edge L 2^-dep) seen from
// squared distance d2: (L 2^-dep)^2 < theta^2 d2 (scalings by powers of two are exact,
// so the forms below decide identically). `meta` is the node's record meta word.
//   bh_accept:   L^2 < theta^2 d2 4^dep (one ldexp of the lane's product);
//   bh_accept_u: L^2 4^-dep < theta^2 d2, the squared edge made from L^2 by lowering its
//                exponent by 2 dep: for a wave-uniform meta that is scalar integer work.
//                Exact because the build accepts only cubes whose L^2 4^-21 is a
//                normal double.
__device__ __forceinline__ bool bh_accept(double L2, double theta2, double d2, uint32_t meta) {
  return L2 < ldexp(theta2 * d2, (int)((meta >> (kSkipBits - 1)) & 62u));
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double edge2_at(double L2, uint32_t meta) {
  u32x2 w = __builtin_bit_cast(u32x2, L2);
  w.y -= ((meta >> kSkipBits) & 31u) << 21;
  return __builtin_bit_cast(double, w);
}

__device__ __forceinline__ bool bh_accept_u(double L2, double theta2, double d2, uint32_t meta) {
  return edge2_at(L2, meta) < theta2 * d2;
}

// The same test as a bound on d2 alone, where theta <= 1/2, every position lies in the
// cube and L^2 < kAcceptL2Max. D = accept_bound(L^2, theta^2) is the largest double with
// fl(theta^2 D) <= L^2; the rounded product is non-decreasing in d2, so the root test
// passes iff d2 > D. At depth dep it passes iff d2 > D 4^-dep: around the bound the
// product is a normal double (at least L^2 4^-21), where scaling by 4^-dep commutes with
// its rounding, and D 4^-21 is normal (D >= 4 L^2). With theta = 0, D = DBL_MAX, and
// DBL_MAX 4^-21 lies far above any d2 between points of a cube with L^2 < 2^900, so
// nothing is accepted, as theta^2 d2 = 0 says. The bound takes the product's place in
// the per-node step, with the same decisions.
constexpr double kAcceptL2Max = 0x1p900;

__host__ __device__ inline double accept_bound(double L2, double theta2) {
  if (!(theta2 > 0.0)) return DBL_MAX;
  double d = L2 / theta2;                // within an ulp or two of the bound
  if (d > DBL_MAX) d = DBL_MAX;
  while (d > 0.0 && theta2 * d > L2) d = nextafter(d, 0.0);
  for (;;) {
    const double up = nextafter(d, DBL_MAX);
    if (up == d || !(theta2 * up <= L2)) break;
    d = up;
  }
  return d;
}

__device__ __forceinline__ bool bh_accept_d(double acc_d2, double d2, uint32_t meta) {
  return edge2_at(acc_d2, meta) < d2;
}

// v * 2^-y with y = d2 * k2 (= v exp(-d2 / sigma^2)), or exactly 0 where `keep` is
// false or exp(-d2 / sigma^2) underflows in float64. Branch-free: the walks evaluate
// it on every lane. A dropped entry gets the exponent -2048, which takes any
// v * mant < 2^31 to 0, so the mask costs one 32-bit select instead of a 64-bit one.
// -floor(y) is the hardware's truncating conversion of -y (y >= 0), which saturates
// out of range; it is used only where y <= kMaxY.
__device__ __forceinline__ double kernel_weight_vd(bool keep, double vd, double d2, double k2) {
  const double y = d2 * k2;
  const double fr = __builtin_amdgcn_fract(y);
  int nfl;
  asm("v_cvt_i32_f64_e64 %0, -%1" : "=v"(nfl) : "v"(y));
  const int e = (keep && y <= kMaxY) ? nfl : -2048;
  const double mant = (double)__builtin_amdgcn_exp2f(-(float)fr);
  return ldexp(vd * mant, e);
}

__device__ __forceinline__ double kernel_weight_if(bool keep, int32_t v, double d2, double k2) {
  return kernel_weight_vd(keep, (double)v, d2, k2);
}

__device__ __forceinline__ double kernel_weight(int32_t v, double d2, double k2) {
  return kernel_weight_if(true, v, d2, k2);
}

struct SumPass {
  double k2;                                      // log2(e) / sigma^2
  double Z = 0.0;
  __device__ __forceinline__ bool operator()(int32_t, bool, int32_t v, double d2) {
    Z = Z + kernel_weight(v, d2, k2);
    return false;
  }
};

// First entry whose running sum exceeds T (same weights, same order as SumPass).
struct SelectPass {
  double k2;
  double T;
  double P = 0.0;
  int32_t chosen = -1;
  bool chosen_neuron = false;
  int32_t last = -1;
  bool last_neuron = false;
  __device__ __forceinline__ bool operator()(int32_t id, bool neuron, int32_t v, double d2) {
    const double w = kernel_weight(v, d2, k2);
    if (w > 0.0) {
      last = id;
      last_neuron = neuron;
    }
    P = P + w;
    if (P > T) {
      chosen = id;
      chosen_neuron = neuron;
      return true;
    }
    return false;
  }
};

__device__ __forceinline__ double dist2(double ax, double ay, double az, double bx, double by,
                                        double bz) {
  const double dx = ax - bx;
  const double dy = ay - by;
  const double dz = az - bz;
  return __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));   // two fused steps
}

// Members of a leaf node x (record r) other than the source, with their counts.
template <class F>
__device__ __forceinline__ bool leaf_entries(const SearchArgs& A, const int32_t* vs, int32_t x,
                                             const NodeRec& r, int32_t i, double xi, double yi,
                                             double zi, F& f) {
  if (!(r.meta & kBucketBit)) {
    const int32_t id = (int32_t)(r.meta & kIdMask);
    if (id == i) return false;
    return f(id, true, r.v, dist2(xi, yi, zi, r.x, r.y, r.z));
  }
  for (int32_t p = A.nbeg[x]; p < A.nend[x]; ++p) {
    const int32_t id = A.order[p];
    const int32_t v = vs[p];
    if (id == i || v == 0) continue;
    const double* q = A.pos + 3 * (int64_t)id;
    if (f(id, true, v, dist2(xi, yi, zi, q[0], q[1], q[2]))) return true;
  }
  return false;
}

// Node records examined and nodes opened (the algorithmic work of one expansion).
struct Count {
  int32_t visits = 0, opens = 0;
  int32_t entries = 0;             // level-0 sweep only: entries of the accepted list
};

// The source's own walk over pre-order positions [x, end) of a start cell's
// subtree (visiting, skipping, opening and accepting as the search rules say).
template <bool COUNT, class F>
__device__ void expand_range(const SearchArgs& A, const NodeRec* __restrict__ R, const int32_t* vs,
                             int32_t x, int32_t end, int32_t i, int32_t li, double xi, double yi,
                             double zi, F& f, Count& cnt) {
  while (x < end) {
    const NodeRec r = R[x];
    if (COUNT) cnt.visits += 1;
    if (r.meta & kLeafBit) {
      if (r.v != 0 && leaf_entries(A, vs, x, r, i, xi, yi, zi, f)) return;
      ++x;
      continue;
    }
    int32_t sk = (int32_t)(r.meta & kSkipMask);
    sk = sk > x ? sk : x + 1;
    if (r.v == 0) {
      x = sk;
      continue;
    }
    if (A.own && li >= x && li < sk) {   // the source's own cell is always opened,
                                         // where the acceptance test could pass it
      if (COUNT) cnt.opens += 1;
      ++x;
      continue;
    }
    const double d2 = dist2(xi, yi, zi, r.x, r.y, r.z);
    if (bh_accept(A.L2, A.theta2, d2, r.meta)) {
      if (f(x, false, r.v, d2)) return;
      x = sk;
    } else {
      if (COUNT) cnt.opens += 1;
      ++x;
    }
  }
}

// Accepted list of the expansion of start node S for source i, in list order.
template <bool COUNT, class F>
__device__ void expand(const SearchArgs& A, const NodeRec* __restrict__ R, const int32_t* vs,
                       int32_t S, int32_t i, int32_t li, double xi, double yi, double zi, F& f,
                       Count& cnt) {
  const NodeRec s = R[S];
  if (COUNT) cnt.visits += 1;
  if (s.meta & kLeafBit) {
    if (s.v != 0) (void)leaf_entries(A, vs, S, s, i, xi, yi, zi, f);
    return;
  }
  if (COUNT) cnt.opens += 1;
  expand_range<COUNT>(A, R, vs, S + 1, (int32_t)(s.meta & kSkipMask), i, li, xi, yi, zi, f, cnt);
}

__device__ __forceinline__ double draw_u(uint64_t seed, int32_t i, int32_t j, uint64_t step,
                                         int level) {
  const uint64_t r = philox_word0(seed, 0, (uint64_t)i, (uint64_t)j, step, (uint64_t)level);
  return (double)(r >> 40) * 0x1p-24;
}

constexpr int32_t kDeferred = -2;      // restart handed on to the second phase
constexpr int kNoDefer = 1 << 20;      // a defer depth no cell reaches

// Depth of an inner node (a drawn cell is always one: leaf entries are neurons).
__device__ __forceinline__ int cell_depth(uint32_t meta) {
  return (int)((meta >> kSkipBits) & 31u);
}

// A restart level's list is short (the children of a far cell, mostly): the sum walk
// keeps up to kRestartKeep entries (weight; id with bit 31 set for a neuron) in
// per-thread memory `stride` elements apart, and the choice is then made from them in
// the same order with the same additions, without a second walk.
constexpr int kRestartKeep = 8;
constexpr uint32_t kKeptNeuron = 0x80000000u;

struct KeptEntries {
  double* w;
  uint32_t* id;
  int stride;
};

struct SumKeepPass {
  double k2;
  KeptEntries K;
  double Z = 0.0;
  int n = 0;
  __device__ __forceinline__ bool operator()(int32_t id, bool neuron, int32_t v, double d2) {
    const double w = kernel_weight(v, d2, k2);
    Z = Z + w;
    if (n < kRestartKeep) {
      K.w[n * K.stride] = w;
      K.id[n * K.stride] = (uint32_t)id | (neuron ? kKeptNeuron : 0u);
    }
    ++n;
    return false;
  }
};

// Levels >= level0 of a search (level0 >= 1): restart at the chosen cell S until a
// neuron is drawn. A cell at depth >= defer_depth is not expanded here: the call
// returns kDeferred with *S_out = that cell and *levels_out = the levels drawn so far
// (its expansion is level *levels_out), for the second phase to continue from.
// keep (nullable): memory for the entries of a level (see SumKeepPass).
template <bool COUNT, bool DEFER>
__device__ int32_t restart_search(const SearchArgs& A, const NodeRec* R, const int32_t* vs,
                                  int32_t S, int level0, int defer_depth, int32_t i, int32_t j,
                                  int32_t li, double xi, double yi, double zi, int* levels_out,
                                  Count& cnt, int32_t* S_out, const KeptEntries* keep = nullptr) {
  Count none;
  for (int level = level0; level < kMaxLevels; ++level) {
    if (DEFER && cell_depth(R[S].meta) >= defer_depth) {
      *S_out = S;
      return kDeferred;
    }
    int32_t id;
    bool neuron;
    if (keep) {
      SumKeepPass s{A.k2, *keep};
      expand<COUNT>(A, R, vs, S, i, li, xi, yi, zi, s, cnt);
      *levels_out = level + 1;
      if (!(s.Z > 0.0)) return -1;
      const double T = draw_u(A.seed, i, j, A.step, level) * s.Z;
      if (s.n <= kRestartKeep) {
        // SelectPass over the kept entries
        double P = 0.0;
        int32_t chosen = -1, last = -1;
        bool chosen_neuron = false, last_neuron = false;
        for (int e = 0; e < s.n; ++e) {
          const double w = keep->w[e * keep->stride];
          const uint32_t r = keep->id[e * keep->stride];
          const int32_t eid = (int32_t)(r & ~kKeptNeuron);
          const bool en = (r & kKeptNeuron) != 0;
          if (w > 0.0) {
            last = eid;
            last_neuron = en;
          }
          P = P + w;
          if (P > T) {
            chosen = eid;
            chosen_neuron = en;
            break;
          }
        }
        id = chosen >= 0 ? chosen : last;
        neuron = chosen >= 0 ? chosen_neuron : last_neuron;
      } else {
        SelectPass p{A.k2, T};
        expand<false>(A, R, vs, S, i, li, xi, yi, zi, p, none);
        id = p.chosen >= 0 ? p.chosen : p.last;
        neuron = p.chosen >= 0 ? p.chosen_neuron : p.last_neuron;
      }
    } else {
      SumPass s{A.k2};
      expand<COUNT>(A, R, vs, S, i, li, xi, yi, zi, s, cnt);
      *levels_out = level + 1;
      if (!(s.Z > 0.0)) return -1;
      const double T = draw_u(A.seed, i, j, A.step, level) * s.Z;
      SelectPass p{A.k2, T};
      expand<false>(A, R, vs, S, i, li, xi, yi, zi, p, none);
      id = p.chosen >= 0 ? p.chosen : p.last;
      neuron = p.chosen >= 0 ? p.chosen_neuron : p.last_neuron;
    }
    if (id < 0) return -1;
    if (neuron) return id;
    S = id;
  }
  atomicOr(A.err, kErrArgs);
  return -1;
}

struct DiagOut {
  double* z0;
  int32_t* levels;
  int32_t* visits;
  int32_t* opens;
  int32_t* visits0;
  int32_t* opens0;
  int32_t* entries0;
};

}  // namespace msp
