// Electrical activity between connectivity updates (Sec. II, "Update of electrical
// activity"), with the firing-rate approximation of Sec. IV-B. One step is 1 ms:
//   * exchange: the spike a source recorded in the previous step reaches the target.
//     Exact synapses are grouped by source once per run (act_setup_k, act_group_k),
//     and a neuron that spikes delivers along its own group into the next step's
//     arrival counts (act_neuron_k; act_deliver_k for the spikes recorded before the
//     run), so a step touches only the synapses of the neurons that fired.
//     Approximated synapses (approx 1: those whose two neurons carry different ranks;
//     approx 2: all) carry a spike at step t iff u < f_i, f_i being the source's
//     frequency over the previous epoch (spikes per step) and u = (Philox word 0 >> 11)
//     2^-53, key (seed, 5), counter (s, t, 0, 0) (act_approx_k, every step, one thread
//     per synapse). Targets count excitatory and inhibitory arrivals (exact integer
//     atomics, so the order of the deliveries does not matter);
//   * neuron model (act_neuron_k, one thread per neuron): Izhikevich 2003, regular
//     spiking (excitatory) or fast spiking (inhibitory):
//       I = w_e e - w_i h + mu + width (u' - 1/2), u' from key (seed, 6), counter (g, t, 0, 0);
//       v += (0.04 v^2 + 5 v + 140 - u + I) / 2, twice (two half-millisecond steps);
//       u += a (b v - u); v >= 30: spike, v = c, u += d;
//   * calcium, a running average of the spikes: Ca -= Ca / tau, then += beta on a spike;
//   * a step t with (t + 1) % delta == 0 closes an epoch: f = spikes in it / delta.
// Only +, -, * and comparisons on fp64 (1/tau and 1/delta come from the host), with
// no contraction, so every value is exactly the IEEE evaluation of these formulas.
#pragma once

#include "common.hpp"

namespace msp {

constexpr int kActBlock = 256;

struct ActParams {
  double a[2], b[2], c[2], d[2];   // per neuron type (0 excitatory, 1 inhibitory)
  double w_e, w_i, mu, width, beta, inv_tau, inv_delta;
  int32_t delta;
};

// Start of the activity (one thread per neuron): the membrane potential at the reset
// value c of the neuron's type, the recovery variable at its resting relation u = b c,
// no calcium, no spike, an empty epoch and no frequency yet.
__global__ void __launch_bounds__(kActBlock) act_init_k(
    int64_t n, const uint8_t* __restrict__ type, ActParams P, double* __restrict__ v,
    double* __restrict__ u, double* __restrict__ calcium, uint8_t* __restrict__ spiked,
    int32_t* __restrict__ count, double* __restrict__ freq, int32_t* err) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const uint8_t t8 = type[g];
  if (t8 > 1) atomicOr(err, 1);
  const int t = t8 ? 1 : 0;
  v[g] = P.c[t];
  u[g] = P.b[t] * P.c[t];
  calcium[g] = 0.0;
  spiked[g] = 0;
  count[g] = 0;
  freq[g] = 0.0;
}

// Run setup, one thread per synapse: a synapse with an endpoint outside [0, n) or a
// type > 1 sets *err and takes no part in the run. Exact synapses are counted per
// source (cnt); with approx 1, remote[s] = 1 marks the approximated ones (neurons of
// different ranks: the two rank gathers are paid once per run, not every step).
__global__ void __launch_bounds__(kActBlock) act_setup_k(
    int64_t n, int64_t m, const int32_t* __restrict__ src, const int32_t* __restrict__ tgt,
    const uint8_t* __restrict__ stype, const int32_t* __restrict__ rank, int32_t approx,
    int32_t* cnt, uint8_t* __restrict__ remote, int32_t* err) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int32_t i = src[s], g = tgt[s];
  const bool ok = i >= 0 && i < n && g >= 0 && g < n && stype[s] <= 1;
  if (!ok) atomicOr(err, 1);
  const bool approxd = approx == 2 || (approx == 1 && ok && rank[i] != rank[g]);
  if (remote) remote[s] = ok && approxd ? 1 : 0;
  if (ok && !approxd) atomicAdd(&cnt[i], 1);
}

// Exact synapses by source: perm[soff[i] .. soff[i + 1]) (cur: zeroed cursors).
__global__ void __launch_bounds__(kActBlock) act_group_k(
    int64_t n, int64_t m, const int32_t* __restrict__ src, const int32_t* __restrict__ tgt,
    const uint8_t* __restrict__ stype, const int32_t* __restrict__ rank, int32_t approx,
    const int32_t* __restrict__ soff, int32_t* cur, int32_t* __restrict__ perm) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int32_t i = src[s], g = tgt[s];
  const bool ok = i >= 0 && i < n && g >= 0 && g < n && stype[s] <= 1;
  const bool approxd = approx == 2 || (approx == 1 && ok && rank[i] != rank[g]);
  if (ok && !approxd) perm[soff[i] + atomicAdd(&cur[i], 1)] = (int32_t)s;
}

// Neuron g's spike along its exact synapses, into the arrival counts e, h.
__device__ __forceinline__ void act_send(int64_t g, const int32_t* __restrict__ soff,
                                         const int32_t* __restrict__ perm,
                                         const int32_t* __restrict__ tgt,
                                         const uint8_t* __restrict__ stype, int32_t* e,
                                         int32_t* h) {
  const int32_t q1 = soff[g + 1];
  for (int32_t q = soff[g]; q < q1; ++q) {
    const int32_t s = perm[q];
    atomicAdd(stype[s] ? &h[tgt[s]] : &e[tgt[s]], 1);
  }
}

// The spikes recorded before the run (spk), delivered for its first step.
__global__ void __launch_bounds__(kActBlock) act_deliver_k(
    int64_t n, const uint8_t* __restrict__ spk, const int32_t* __restrict__ soff,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ tgt,
    const uint8_t* __restrict__ stype, int32_t* e, int32_t* h) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n || !spk[g]) return;
  act_send(g, soff, perm, tgt, stype, e, h);
}

// The approximated synapses of approx 1, packed in synapse order (pos: exclusive scan
// of remote): their index (the draw's counter), endpoints and type.
__global__ void __launch_bounds__(kActBlock) act_pack_k(
    int64_t m, const int32_t* __restrict__ src, const int32_t* __restrict__ tgt,
    const uint8_t* __restrict__ stype, const uint8_t* __restrict__ remote,
    const int32_t* __restrict__ pos, int32_t* __restrict__ aidx, int32_t* __restrict__ asrc,
    int32_t* __restrict__ atgt, uint8_t* __restrict__ atype) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m || !remote[s]) return;
  const int32_t q = pos[s];
  aidx[q] = (int32_t)s;
  asrc[q] = src[s];
  atgt[q] = tgt[s];
  atype[q] = stype[s];
}

// Approximated synapses at step t: the packed list of approx 1 (aidx non-null, count
// *na), or every synapse with valid endpoints (approx 2).
__global__ void __launch_bounds__(kActBlock) act_approx_k(
    int64_t n, int64_t m, const int32_t* __restrict__ src, const int32_t* __restrict__ tgt,
    const uint8_t* __restrict__ stype, const int32_t* __restrict__ aidx,
    const int32_t* __restrict__ na, uint64_t seed, uint64_t t, const double* __restrict__ freq,
    int32_t* e, int32_t* h) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (aidx ? (int64_t)*na : m)) return;
  const int32_t i = src[q], g = tgt[q];
  const uint8_t ty = stype[q];
  if (i < 0 || i >= n || g < 0 || g >= n || ty > 1) return;     // reported at setup
  const uint64_t s = aidx ? (uint64_t)aidx[q] : (uint64_t)q;
  const double u = (double)(philox_word0(seed, 5, s, t, 0, 0) >> 11) * 0x1p-53;
  if (u < freq[i]) atomicAdd(ty ? &h[g] : &e[g], 1);
}

// The step's arrivals e, h are consumed (and cleared for the step after next) here; a
// neuron that fires sends along its exact synapses into the next step's e2, h2 (soff
// null: no exact synapses).
__global__ void __launch_bounds__(kActBlock) act_neuron_k(
    int64_t n, const uint8_t* __restrict__ ntype, ActParams P, uint64_t seed, uint64_t t,
    double* __restrict__ v, double* __restrict__ u, double* __restrict__ ca,
    uint8_t* __restrict__ spk, int32_t* __restrict__ count, double* __restrict__ freq,
    int32_t* __restrict__ e, int32_t* __restrict__ h, int32_t* __restrict__ last_input,
    int64_t* __restrict__ part, const int32_t* __restrict__ soff,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ tgt,
    const uint8_t* __restrict__ stype, int32_t* e2, int32_t* h2) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool f = false;
  if (g < n) {
    const int k = ntype[g] ? 1 : 0;
    const int32_t ne = e[g], nh = h[g];
    e[g] = 0;
    h[g] = 0;
    if (last_input) {
      last_input[g] = ne;
      last_input[n + g] = nh;
    }
    const double uu = (double)(philox_word0(seed, 6, (uint64_t)g, t, 0, 0) >> 11) * 0x1p-53;
    const double I = P.w_e * (double)ne - P.w_i * (double)nh + (P.mu + P.width * (uu - 0.5));
    double vv = v[g], w = u[g];
    vv = vv + 0.5 * (0.04 * vv * vv + 5.0 * vv + 140.0 - w + I);
    vv = vv + 0.5 * (0.04 * vv * vv + 5.0 * vv + 140.0 - w + I);
    w = w + P.a[k] * (P.b[k] * vv - w);
    f = vv >= 30.0;
    if (f) {
      vv = P.c[k];
      w = w + P.d[k];
    }
    v[g] = vv;
    u[g] = w;
    double c = ca[g];
    c = c - c * P.inv_tau;
    if (f) c = c + P.beta;
    ca[g] = c;
    spk[g] = f ? 1 : 0;
    if (f && soff) act_send(g, soff, perm, tgt, stype, e2, h2);
    int32_t cnt = count[g] + (f ? 1 : 0);
    if ((t + 1) % (uint64_t)P.delta == 0) {
      freq[g] = (double)cnt * P.inv_delta;
      cnt = 0;
    }
    count[g] = cnt;
  }
  if (part) {                       // this block's spikes, added to its own slot
    __shared__ int32_t wave_spikes[kActBlock / 64];
    const uint64_t b = __ballot(f);
    if ((threadIdx.x & 63) == 0) wave_spikes[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t sum = 0;
      for (int w = 0; w < kActBlock / 64; ++w) sum += wave_spikes[w];
      part[blockIdx.x] += sum;
    }
  }
}

// Sum of the per-block spike counts, added to *spikes (one block).
__global__ void __launch_bounds__(kActBlock) act_spikes_k(const int64_t* __restrict__ part,
                                                         int64_t nblocks, int64_t* spikes) {
  __shared__ int64_t acc[kActBlock];
  int64_t sum = 0;
  for (int64_t q = threadIdx.x; q < nblocks; q += kActBlock) sum += part[q];
  acc[threadIdx.x] = sum;
  __syncthreads();
  for (int w = kActBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) acc[threadIdx.x] += acc[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *spikes += acc[0];
}

}  // namespace msp
