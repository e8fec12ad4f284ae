// One connectivity update after the search (Sec. III-A, "Update of synapses" and
// "Update of synaptic elements"), enqueued as kernels only: the request acceptance
// (commit), the recording of the new synapses, and the plasticity step (growth,
// deletion, retraction, vacancies). Every count the sequence needs (requests,
// synapses, retraction candidates, survivors) may be known on the host or only on the
// device (DevCount); nothing is read back and nothing is allocated, so the same
// sequence serves the host entry points (which then read their status once) and the
// update cycle (msp_cycle), which captures it in a graph.
#pragma once

#include "commit.hpp"
#include "plasticity.hpp"
#include "scan.hpp"

namespace msp {

// ---------------------------------------------------------------------------- commit
// Working memory of the acceptance of up to `cap_S` requests among n neurons.
struct CommitWs {
  int32_t* src_of;
  int64_t* key;
  uint64_t* prio;
  int32_t* cnt;                 // [2n] requests per group, then the accepted ones
  int32_t* within;              // [cap_S] each request's place in its group
  GroupThr* thr;                // [2n] each group's decision
  int32_t* seg_off;             // [2n + 1]
  int32_t* seg;
  uint8_t* acc;
  int64_t* dst;                 // [cap_S + 1]
  int32_t* flags;               // [1] kErrArgs, kCommitCapacity
  void* scan_ws;
};

inline CommitWs commit_ws(void* base, int64_t n, int64_t cap_S, size_t* bytes) {
  Carver c{static_cast<char*>(base)};
  CommitWs w;
  w.src_of = c.take<int32_t>(cap_S);
  w.key = c.take<int64_t>(cap_S);
  w.prio = c.take<uint64_t>(cap_S);
  w.cnt = c.take<int32_t>(2 * n);
  w.within = c.take<int32_t>(cap_S);
  w.thr = c.take<GroupThr>(2 * n);
  w.seg_off = c.take<int32_t>(2 * n + 1);
  w.seg = c.take<int32_t>(cap_S);
  w.acc = c.take<uint8_t>(cap_S);
  w.dst = c.take<int64_t>(cap_S + 1);
  w.flags = c.take<int32_t>(1);
  w.scan_ws = c.take_bytes(std::max(scan_tmp_bytes<int32_t>(2 * n),
                                    scan_tmp_bytes<int64_t>(cap_S + 1)));
  *bytes = c.off;
  return w;
}

// The S requests (slots of `target` in (source, element) order; elem_offset [n + 1])
// compete per (target, type) group for its vacancies; the accepted ones become
// synapses at syn_* [0, *n_formed) and take one vacancy of each side. If the accepted
// requests exceed syn_capacity, or a target is >= n, nothing is written and
// *n_formed = 0 (w.flags says which).
inline hipError_t enqueue_commit(const CommitWs& w, const int32_t* target,
                                 const int64_t* elem_offset, const uint8_t* neuron_type,
                                 int64_t n, DevCount S, int32_t* vac_axon, int32_t* vac_exc,
                                 int32_t* vac_inh, uint64_t seed, DevStep step, int32_t* syn_src,
                                 int32_t* syn_tgt, uint8_t* syn_type, int64_t syn_capacity,
                                 int64_t* n_formed, uint8_t* accepted_out, hipStream_t s) {
  const unsigned gs = grid_cap(S.v, kCommitBlock);
  fill_i32_k<<<grid_for(2 * n, 256), 256, 0, s>>>(w.cnt, 2 * n, 0);
  fill_i32_k<<<1, 64, 0, s>>>(w.flags, 1, 0);
  src_of_k<<<grid_for(n, kCommitBlock), kCommitBlock, 0, s>>>(elem_offset, n, S, w.src_of);
  req_key_k<<<gs, kCommitBlock, 0, s>>>(target, elem_offset, w.src_of, neuron_type, S, n, seed,
                                        step, w.key, w.prio, w.cnt, w.within, w.flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = exclusive_scan<int32_t, int32_t, Ident<int32_t>>(w.cnt, w.seg_off, 2 * n, Ident<int32_t>(),
                                                       true, s, w.scan_ws);
  if (e != hipSuccess) return e;
  req_scatter_k<<<gs, kCommitBlock, 0, s>>>(w.key, S, w.seg_off, w.within, w.seg);
  // decisions per group (w.cnt now takes each group's accepted count), then per request
  const unsigned gg = grid_cap(2 * n, kCommitBlock);
  group_thr_k<<<gg, kCommitBlock, 0, s>>>(w.prio, w.seg_off, w.seg, 2 * n, vac_exc, vac_inh,
                                          w.thr, w.cnt);
  req_decide_k<<<gs, kCommitBlock, 0, s>>>(w.key, w.prio, w.thr, w.seg_off, w.seg, S, vac_exc,
                                           vac_inh, w.acc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = exclusive_scan<int64_t, uint8_t, AccFlag>(w.acc, w.dst, S.v, AccFlag(), true, s, w.scan_ws,
                                                S.p);
  if (e != hipSuccess) return e;
  commit_write_k<<<gs, kCommitBlock, 0, s>>>(w.acc, w.dst, w.key, w.src_of, S, syn_capacity,
                                             syn_src, syn_tgt, syn_type, accepted_out, w.flags);
  dec_groups_k<<<gg, kCommitBlock, 0, s>>>(w.cnt, 2 * n, w.dst, S, syn_capacity, w.flags,
                                           vac_exc, vac_inh);
  dec_sources_k<<<grid_cap(n, kCommitBlock), kCommitBlock, 0, s>>>(
      elem_offset, n, w.acc, w.dst, S, syn_capacity, w.flags, vac_axon);
  formed_k<<<1, 64, 0, s>>>(w.dst, S, syn_capacity, w.flags, n_formed);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------- plasticity
struct PlastConst {
  double ca_mean, ca_sd, xi, zeta, scale;   // growth rule (see growth_k)
  double delete_fraction;
};

// Working memory of a plasticity step over a list of up to cap_m synapses.
struct PlastWs {
  uint8_t* dead;
  uint8_t* cflag;               // retraction candidates of one kind
  uint64_t* k0;
  uint64_t* k1;
  int32_t* v0;
  int32_t* v1;
  int32_t* pos;                 // [cap_m + 1]
  int32_t* exc;                 // [n]
  void* sort_ws;
  void* scan_ws;
  SynList O;                    // the survivors, compacted
  DelSelect* st;
  uint32_t* hist;               // [256]
  int64_t* cnt;                 // [2] retraction candidates, survivors
  int32_t* cnt32;               // [1] retraction candidates (the sort's count)
};

inline PlastWs plast_ws(void* base, int64_t n, int64_t cap_m, size_t* bytes) {
  Carver c{static_cast<char*>(base)};
  PlastWs w;
  w.dead = c.take<uint8_t>(cap_m);
  w.cflag = c.take<uint8_t>(cap_m);
  w.k0 = c.take<uint64_t>(cap_m);
  w.k1 = c.take<uint64_t>(cap_m);
  w.v0 = c.take<int32_t>(cap_m);
  w.v1 = c.take<int32_t>(cap_m);
  w.pos = c.take<int32_t>(cap_m + 1);
  w.exc = c.take<int32_t>(n);
  w.sort_ws = c.take_bytes(radix_sort_ws_bytes(cap_m));
  w.scan_ws = c.take_bytes(scan_tmp_bytes<int32_t>(cap_m + 1));
  w.O.src = c.take<int32_t>(cap_m);
  w.O.tgt = c.take<int32_t>(cap_m);
  w.O.type = c.take<uint8_t>(cap_m);
  w.st = c.take<DelSelect>(1);
  w.hist = c.take<uint32_t>(256);
  w.cnt = c.take<int64_t>(2);
  w.cnt32 = c.take<int32_t>(1);
  *bytes = c.off;
  return w;
}

// Growth, deletion and retraction over the m synapses of L, then the vacancies
// (plasticity.hpp states the rules). The survivors keep their order; their count goes
// to *m_out (which may be m's own device count: it is written last).
inline hipError_t enqueue_plasticity(const PlastWs& w, int64_t n, const PlastConst& c,
                                     uint64_t seed, DevStep step, double* z, int32_t* bound,
                                     SynList L, DevCount m, int64_t* m_out, int32_t* vac_axon,
                                     int32_t* vac_exc, int32_t* vac_inh, hipStream_t s) {
  growth_k<<<grid_for(3 * n, kPlastBlock), kPlastBlock, 0, s>>>(z, n, seed, step, c.ca_mean,
                                                               c.ca_sd, c.xi, c.zeta, c.scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (m.v > 0) {
    const unsigned gm = grid_cap(m.v, kPlastBlock);
    fill_u8_k<<<gm, kPlastBlock, 0, s>>>(w.dead, m, 0);
    if (c.delete_fraction > 0.0) {
      // the round(frac m) synapses of smallest (priority, index): a radix selection of
      // the threshold key, most significant digit first, then one marking pass
      del_keys_k<<<gm, kPlastBlock, 0, s>>>(w.k0, w.v0, m, seed, step);
      del_select_init_k<<<1, 256, 0, s>>>(w.st, c.delete_fraction, m, w.hist);
      for (int shift = 56; shift >= 0; shift -= 8) {
        del_select_hist_k<<<gm, kPlastBlock, 0, s>>>(w.k0, m, w.st, shift, w.hist);
        del_select_pick_k<<<1, 256, 0, s>>>(w.st, w.hist, shift);
      }
      e = exclusive_scan<int32_t, uint64_t, DelTie>(w.k0, w.pos, m.v, DelTie{w.st}, false, s,
                                                     w.scan_ws, m.p);
      if (e != hipSuccess) return e;
      del_select_mark_k<<<gm, kPlastBlock, 0, s>>>(w.k0, m, w.st, w.pos, L, n, w.dead, bound);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    int owner_bits = 1;
    while (owner_bits < 31 && ((int64_t)1 << owner_bits) < n) ++owner_bits;
    const int key_bits = (32 + owner_bits + 7) / 8 * 8;
    const DevCount C{m.v, w.cnt};
    for (int k = 0; k < 3; ++k) {
      excess_k<<<grid_for(n, kPlastBlock), kPlastBlock, 0, s>>>(bound + k * n, z + k * n, n,
                                                               w.exc);
      const RetractFlag F{L, w.dead, w.exc, k};
      retract_flag_k<<<gm, kPlastBlock, 0, s>>>(F, m, w.cflag);
      e = exclusive_scan<int32_t, uint8_t, ByteCount>(w.cflag, w.pos, m.v, ByteCount(), true, s,
                                                      w.scan_ws, m.p);
      if (e != hipSuccess) return e;
      take_count_k<<<1, 64, 0, s>>>(w.pos, m, w.cnt, w.cnt32);
      cand_write_k<<<gm, kPlastBlock, 0, s>>>(F, w.pos, m, seed, step, w.k0, w.v0);
      e = radix_sort_pairs_ws(w.k0, w.v0, w.k1, w.v1, m.v, key_bits, s, w.sort_ws, w.cnt32);
      if (e != hipSuccess) return e;
      retract_k<<<gm, kPlastBlock, 0, s>>>(w.k0, w.v0, C, w.exc, L, n, w.dead, bound);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    e = exclusive_scan<int32_t, int32_t, LiveFlag>(nullptr, w.pos, m.v, LiveFlag{w.dead}, true, s,
                                                   w.scan_ws, m.p);
    if (e != hipSuccess) return e;
    take_count_k<<<1, 64, 0, s>>>(w.pos, m, w.cnt + 1, nullptr);
    compact_k<<<gm, kPlastBlock, 0, s>>>(L, w.dead, w.pos, m, w.O);
    copy_list_k<<<gm, kPlastBlock, 0, s>>>(w.O, DevCount{m.v, w.cnt + 1}, L);
    copy_scalar_k<<<1, 64, 0, s>>>(w.cnt + 1, m_out);
  } else {
    fill_i64_k<<<1, 64, 0, s>>>(m_out, 1, 0);
  }
  vacancy_k<<<grid_for(3 * n, kPlastBlock), kPlastBlock, 0, s>>>(z, bound, n, vac_axon, vac_exc,
                                                                vac_inh);
  return hipGetLastError();
}

}  // namespace msp
