// Expected attraction and its adjoint (the differentiated form of the search).
//
// For a source i with vacant axonal elements, Z_i is the normaliser of its level-0
// list: the sum over the accepted entries e (cells and neurons, type of i) of
// w_e = v_e exp(-|x_i - c_e|^2 / sigma^2). Given upstream gradients g_i = dLoss/dZ_i,
// with every acceptance decision held at the current geometry:
//   dZ_i/dx_i     = sum_e w_e * (-2 (x_i - c_e) / sigma^2)
//   dZ_i/dc_e     = w_e * 2 (x_i - c_e) / sigma^2        (a neuron entry: c_e = x_j)
//   dZ_i/dsigma   = sum_e w_e * 2 |x_i - c_e|^2 / sigma^3
//   dc_C/dx_j     = (v_j / v_C) I for every neuron j of cell C (a centroid is the
//                   vacancy-weighted mean of its neurons).
// The forward pass is the search's level-0 sweep without checkpoints (Z per source).
// The backward sweep walks the sources' lists coherently (as the search does); per
// node, the contributions of all lanes of the wave are summed across the wave first
// and added to the node's gradient G with one float64 atomic per component. A
// neuron's leaf is a node like any other (its centroid is the neuron's position), so
// leaves need no separate path. The waves of each die add into that die's own copy
// of G, so the atomics of concurrent waves on the nodes they all share (the upper
// tree) are spread over eight addresses instead of queueing on one; a reduction
// sums the copies. A top-down pass then carries sum_{C containing j} G_C / v_C to
// each neuron.
#pragma once

#include "batch.hpp"

namespace msp {

constexpr int kGradCopies = 8;  // one per die (XCC)

struct AttractArgs {
  const float* gZ;              // [n] upstream gradient, by neuron id
  double* G;                    // [kGradCopies][2][N][3] per-node centroid gradients
  double* dpos;                 // [n][3] float64 accumulator
  double* dsigma;               // scalar accumulator
  double two_over_s2;           // 2 / sigma^2
  double two_over_s3;           // 2 / sigma^3
  int64_t N;
  const int32_t* unit_count;    // device scalar: the sweep units (parts of tiles)
};

// The die (XCC) this wave runs on: bits 3:0 of hardware register XCC_ID (20). It only
// selects a copy of G; any value in 0..7 gives the same sums.
__device__ __forceinline__ int xcc_id() {
  return (int)(__builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & (kGradCopies - 1));
}



// v moved across lanes by a DPP pattern (both 32-bit halves); lanes of rows outside
// row_mask get 0.0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of the wave (every lane active), returned to every lane. DPP
// steps: pairs, quads (quad_perm), halves of a row (row_half_mirror), rows of 16
// (row_mirror); then rows 0+1 and 2+3 (row_bcast:15), all four (row_bcast:31), which
// leaves the total in lane 63.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1, 0xF>(v);        // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E, 0xF>(v);        // quad_perm [2,3,0,1]
  v += dpp_f64<0x141, 0xF>(v);       // row_half_mirror
  v += dpp_f64<0x140, 0xF>(v);       // row_mirror
  v += dpp_f64<0x142, 0xA>(v);       // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);       // row_bcast:31 into rows 2 and 3
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// v from lane (lane ^ m), through the LDS crossbar (both 32-bit halves).
__device__ __forceinline__ double shfl_xor_f64(double v, int lane, int m) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int addr = (lane ^ m) << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)b);
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// The wave sums of three values at once (every lane active): the lanes split the
// values between them as they add, so each exchange moves one or two values instead of
// three. After the pair and quad steps lane l holds a partial sum of value
// {0, 2, 1, 3}[l % 4] (value 3 is zero), then the four lanes of a row with that value
// and the four rows are added. Returns lane l's full sum of that value; `comp` is set
// to its index (3: none).
__device__ __forceinline__ double wave_sum3(double fx, double fy, double fz, int lane, int& comp) {
  const bool odd = lane & 1;
  // pairs: even lanes keep (x, y) and send (z, 0); odd lanes the other way round
  const double s0 = odd ? fx : fz, s1 = odd ? fy : 0.0;
  const double k0 = odd ? fz : fx, k1 = odd ? 0.0 : fy;
  const double p = k0 + dpp_f64<0xB1, 0xF>(s0);      // quad_perm [1,0,3,2]
  const double q = k1 + dpp_f64<0xB1, 0xF>(s1);
  // quads: lanes 0, 1 of a quad keep p (x, z), lanes 2, 3 keep q (y, 0)
  const bool up = (lane >> 1) & 1;
  double v = (up ? q : p) + dpp_f64<0x4E, 0xF>(up ? p : q);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x124, 0xF>(v);                       // row_ror:4
  v += dpp_f64<0x128, 0xF>(v);                       // row_ror:8
  v += shfl_xor_f64(v, lane, 16);
  v += shfl_xor_f64(v, lane, 32);
  const int r = lane & 3;
  comp = r == 0 ? 0 : r == 1 ? 2 : r == 2 ? 1 : 3;
  return v;
}

// Add the wave's contributions (fx, fy, fz) to dst[0..2] (skipped if
// all are zero).
__device__ __forceinline__ void wave_add3(double fx, double fy, double fz, double* dst, int lane) {
  if (!__any(fx != 0.0 || fy != 0.0 || fz != 0.0)) return;
  int comp = 3;
  const double v = wave_sum3(fx, fy, fz, lane, comp);
  if (lane < 3) atomicAdd(dst + comp, v);
}

// Part `part` of the tile's 2^plog parts (the search's level-0 sweep cut into parts:
// the lane states at the part's first node come from its ancestors).
__device__ void attract_tile(const SearchArgs& A, const AttractArgs& O, int tile, int part,
                             int plog, int lane) {
  const int64_t slot = (int64_t)tile * kWave + lane;
  const int32_t i = A.work[slot];
  const bool valid = i >= 0;
  const int32_t i0 = __builtin_amdgcn_readfirstlane(i);
  const int t = A.type[i0] ? 1 : 0;
  const cptr<NodeRec> R = as_const(A.rec[t]);
  int32_t li = -1;
  double xi = 0.0, yi = 0.0, zi = 0.0, g = 0.0;
  if (valid) {
    li = A.leaf_of[i];
    xi = A.pos[3 * (int64_t)i];
    yi = A.pos[3 * (int64_t)i + 1];
    zi = A.pos[3 * (int64_t)i + 2];
    g = (double)O.gZ[i];
  }
  double dxi = 0.0, dyi = 0.0, dzi = 0.0, ds = 0.0;
  double* G = O.G + ((int64_t)xcc_id() * 2 + t) * O.N * 3;
  // one accepted entry of this lane: the gradient factor f = g * w * 2 / sigma^2
  // applied to the offset (x_i - c)
  auto take = [&](bool on, int32_t v, double cx, double cy, double cz, double& fx, double& fy,
                  double& fz) {
    fx = fy = fz = 0.0;
    if (!on) return;
    const double dx = xi - cx, dy = yi - cy, dz = zi - cz;
    const double d2 = dist2(xi, yi, zi, cx, cy, cz);
    const double w = kernel_weight(v, d2, A.k2);
    const double f = g * w * O.two_over_s2;
    fx = f * dx;
    fy = f * dy;
    fz = f * dz;
    dxi -= fx;
    dyi -= fy;
    dzi -= fz;
    ds += g * w * d2 * O.two_over_s3;
  };
  const NodeRec root = load_rec(R, 0);
  if (!(root.meta & kLeafBit)) {
    const int32_t root_end = (int32_t)(root.meta & kSkipMask);
    int32_t x = 1, end = root_end;
    int32_t me = valid ? 0 : 0x7FFFFFFF;
    if (plog > 0) {
      part_range(li, valid, lane, plog, part, root_end, x, end);
      if (x > 1 && x < end) me = mask_at<true>(A, R, x, me, li, xi, yi, zi);
    }
    while (x < end) {
      const NodeRec cur = load_rec(R, x);
      const bool active = x >= me;
      const uint32_t meta = cur.meta;
      if (meta & kLeafBit) {
        if (cur.v != 0) {
          if (!(meta & kBucketBit)) {
            // a neuron's leaf: its gradient reaches the neuron through the push-down
            const int32_t id = (int32_t)(meta & kIdMask);
            double fx, fy, fz;
            take(active && id != i, cur.v, cur.x, cur.y, cur.z, fx, fy, fz);
            wave_add3(fx, fy, fz, G + 3 * (int64_t)x, lane);
          } else {
            // members of a bucket are entries at their own positions
            const cptr<int32_t> vs = as_const(A.vs[t]);
            const cptr<int32_t> order = as_const(A.order);
            const cptr<double> pos = as_const(A.pos);
            const int32_t pe = as_const(A.nend)[x];
            for (int32_t p = as_const(A.nbeg)[x]; p < pe; ++p) {
              const int32_t id = order[p];
              const int32_t v = vs[p];
              double fx, fy, fz;
              take(active && id != i && v != 0, v, pos[3 * (int64_t)id], pos[3 * (int64_t)id + 1],
                   pos[3 * (int64_t)id + 2], fx, fy, fz);
              wave_add3(fx, fy, fz, O.dpos + 3 * (int64_t)id, lane);
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
      const bool contains = A.own && li >= x && li < sk;
      const double d2 = dist2(xi, yi, zi, cur.x, cur.y, cur.z);
      const bool acc_ok = bh_accept_u(A.L2, A.theta2, d2, meta);
      const bool open = active && (contains || !acc_ok);
      const bool accept = active && !contains && acc_ok;
      double fx, fy, fz;
      take(accept, cur.v, cur.x, cur.y, cur.z, fx, fy, fz);
      wave_add3(fx, fy, fz, G + 3 * (int64_t)x, lane);
      if (accept) me = sk;
      x = __any(open) ? x + 1 : sk;
    }
  }
  if (valid) {
    atomicAdd(O.dpos + 3 * (int64_t)i + 0, dxi);
    atomicAdd(O.dpos + 3 * (int64_t)i + 1, dyi);
    atomicAdd(O.dpos + 3 * (int64_t)i + 2, dzi);
  }
  ds = wave_sum(ds);
  if (lane == 0 && ds != 0.0) atomicAdd(O.dsigma, ds);
}

// One wave per unit, a part of a tile of the batch path's worklist of sources with
// a_i > 0 (one simulation).
__global__ void __launch_bounds__(256) attract_bwd_k(BatchDev B, AttractArgs O) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t unit = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (unit >= *O.unit_count) return;
  const SearchArgs A = args_of(B.sims, 0, B.work);
  const int plog = __builtin_amdgcn_readfirstlane((int)as_const(B.plog)[0]);
  const int local = __builtin_amdgcn_readfirstlane((int)(unit - as_const(B.unit_base)[0]));
  const int tile = as_const(B.tile_base)[0] + (local >> plog);
  attract_tile(A, O, tile, local & ((1 << plog) - 1), plog, lane);
}

// Z of every source from the sweep's part sums (added in part order, then rounded to
// float32); other neurons keep 0.
__global__ void z_scatter_k(BatchDev B, SweepOut W, float* __restrict__ Z) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tile = slot / kWave;
  if (tile >= *W.tile_count) return;
  const int32_t i = B.work[slot];
  if (i < 0) return;
  const int sim = find_sim(B.tile_base, B.nsims, tile);
  const int plog = B.plog[sim];
  const int64_t u0 = (int64_t)B.unit_base[sim] + ((tile - (int64_t)B.tile_base[sim]) << plog);
  const int64_t lane = slot % kWave;
  double z = 0.0;
  for (int q = 0; q < (1 << plog); ++q) z = z + W.Z[(u0 + q) * kWave + lane];
  Z[i] = (float)z;
}

// G = sum of the per-die copies, in die order.
__global__ void grad_sum_k(double* __restrict__ G, int64_t count) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  double s = G[k];
  for (int c = 1; c < kGradCopies; ++c) s += G[(int64_t)c * count + k];
  G[k] = s;
}

__global__ void fill_f64_k(double* p, int64_t n, double v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// Top-down: H(child) = H(node) + G(child) / v(child), per type; the root's H is
// G(root) / v(root) (zero: the root is never accepted). One launch per depth.
__global__ void push_level_k(const int32_t* __restrict__ nodes, int64_t cnt,
                             const NodeRec* __restrict__ r0, const NodeRec* __restrict__ r1,
                             const double* __restrict__ G, double* __restrict__ H, int64_t N) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= cnt) return;
  const int32_t x = nodes[q];
  const uint32_t meta = r0[x].meta;
  if (meta & kLeafBit) return;
  const int32_t end = (int32_t)(meta & kSkipMask);
  for (int t = 0; t < 2; ++t) {
    const NodeRec* r = t ? r1 : r0;
    const double* Gt = G + (int64_t)t * N * 3;
    double* Ht = H + (int64_t)t * N * 3;
    const double hx = Ht[3 * (int64_t)x], hy = Ht[3 * (int64_t)x + 1], hz = Ht[3 * (int64_t)x + 2];
    int32_t c = x + 1;
    while (c < end) {
      const NodeRec rc = r[c];
      double ax = hx, ay = hy, az = hz;
      if (rc.v > 0) {
        const double iv = 1.0 / (double)rc.v;
        ax += Gt[3 * (int64_t)c] * iv;
        ay += Gt[3 * (int64_t)c + 1] * iv;
        az += Gt[3 * (int64_t)c + 2] * iv;
      }
      Ht[3 * (int64_t)c] = ax;
      Ht[3 * (int64_t)c + 1] = ay;
      Ht[3 * (int64_t)c + 2] = az;
      c = (rc.meta & kLeafBit) ? c + 1 : (int32_t)(rc.meta & kSkipMask);
    }
  }
}

// Neurons: dpos_j += sum_t v_j^t H^t(leaf of j); then convert to float32.
__global__ void push_leaves_k(const int32_t* __restrict__ leaf_of, const int32_t* __restrict__ nbeg,
                              const int32_t* __restrict__ nend, const int32_t* __restrict__ order,
                              const int32_t* __restrict__ vs0, const int32_t* __restrict__ vs1,
                              const double* __restrict__ H, int64_t N, int64_t n,
                              const double* __restrict__ dpos64, float* __restrict__ dpos) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int32_t x = leaf_of[j];
  // the neuron's position in sorted order, to read its per-type counts
  int32_t p = nbeg[x];
  while (p < nend[x] && order[p] != (int32_t)j) ++p;
  double a[3] = {dpos64[3 * j], dpos64[3 * j + 1], dpos64[3 * j + 2]};
  for (int t = 0; t < 2; ++t) {
    const int32_t v = t ? vs1[p] : vs0[p];
    if (v <= 0) continue;
    const double* Ht = H + (int64_t)t * N * 3 + 3 * (int64_t)x;
    for (int k = 0; k < 3; ++k) a[k] += (double)v * Ht[k];
  }
  for (int k = 0; k < 3; ++k) dpos[3 * j + k] = (float)a[k];
}

}  // namespace msp
