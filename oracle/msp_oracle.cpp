// TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, fp64 CPU oracle of the MSP connectivity update (arXiv 2509.26193,
// "I Like To Move It"). It exists to check the HIP library; it is called only by
// the tests, by the smoke check and by the benchmark's CPU-baseline leg. It shares
// no code, header or table with the HIP library.
//
// What each function follows in the paper:
//   * octree: Sec. III-B, "Spatial octree" paragraph (root = domain, eight octants,
//     subdivide until a leaf holds at most one neuron) and "Division of the
//     simulation domain" (Morton-indexed cells).
//   * aggregation: Sec. III-B, "Division of work" paragraph (leaf = neuron position
//     and count; inner node = sum of children, position = weighted average of the
//     children; refreshed bottom-up before each connectivity update, which is how Alg. 1
//     begins).
//   * search: Sec. III-A "Update of synapses" (each vacant axonal element scores
//     partners with a distance kernel and draws one) and Sec. III-B "Division of
//     work" (acceptance test cell length / distance < theta, which always rejects the
//     root; rejected nodes are replaced by their children; one node of the accepted
//     list is drawn by probability; an inner node restarts the search there).
//     Sec. II: theta = 0 gives the direct solution.
//   * commit: Sec. III-A "Update of synapses" (neurons accept as many requests as
//     their vacant dendritic elements allow, chosen randomly, and decline the rest)
//     and Sec. III-B (all requests are formed before the exchange).
//   * electrical activity: Sec. II "Update of electrical activity" (exchange the
//     previous step's spikes, new state from the inputs and background noise, record
//     spikes, update calcium, a running average of the firing rate) with the neuron
//     model the paper names (Izhikevich), and Sec. IV-B (between processes, a spike
//     is drawn from the sender's frequency of the previous epoch).
//   * Philox4x64-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
//     as 1, 2, 3", SC'11. The paper leaves the generator open.
//
// Readings where the paper is silent (kernel exp(-d^2/sigma^2), strict "<", cell
// length = cube edge L/2^k, autapses excluded, depth cap 21 with bucket leaves,
// octant digit 4x+2y+z, draws u = top 24 bits of Philox word 0, priorities for the
// random acceptance) are listed with the design notes of the repository. The paper
// prints no value that fixes the kernel's form, so that reading is parity unpinned
// with respect to the paper; every function here is pinned to its own definition by
// the CPU tests (brute force, closed forms, invariants, published known answers).
//
// Build: g++ -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math), so every
// expression is evaluated exactly as written, one rounding per operation.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128 multiplies
// with a Weyl-sequence key schedule.
// ---------------------------------------------------------------------------
struct P4 { uint64_t v[4]; };

P4 philox4x64_10(P4 ctr, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    unsigned __int128 p0 = (unsigned __int128)M0 * ctr.v[0];
    unsigned __int128 p1 = (unsigned __int128)M1 * ctr.v[2];
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    P4 o;
    o.v[0] = hi1 ^ ctr.v[1] ^ k0;
    o.v[1] = lo1;
    o.v[2] = hi0 ^ ctr.v[3] ^ k1;
    o.v[3] = lo0;
    ctr = o;
  }
  return ctr;
}

// u in [0,1): the top 24 bits of word 0, scaled by 2^-24 (exact in fp32 and fp64).
double draw_u(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
  P4 ctr = {{a, b, c, d}};
  P4 r = philox4x64_10(ctr, seed, stream);
  return (double)(r.v[0] >> 40) * 0x1p-24;
}

const int kMaxDepth = 21;           // 21 bits per axis, 63-bit keys
const double kCells = 2097152.0;     // 2^21

}  // namespace

// ---------------------------------------------------------------------------
// Tree
// ---------------------------------------------------------------------------
struct OracleNode {
  int depth;
  uint64_t prefix;          // key >> (63 - 3*depth)
  int64_t begin, end;       // range in the (key, id)-sorted neuron order
  bool leaf;
  std::vector<int64_t> children;   // node indices, octant-digit order
  int64_t subtree_end;      // one past the last pre-order index of the subtree
};

struct OracleTree {
  int64_t n = 0;
  double x0[3] = {0, 0, 0};
  double L = 1;
  std::vector<double> pos;          // [n][3] by neuron id
  std::vector<uint64_t> key;        // by neuron id
  std::vector<int64_t> order;       // neuron ids sorted by (key, id)
  std::vector<OracleNode> nodes;    // pre-order
  // per-type aggregates, refreshed by oracle_update_counts
  std::vector<int64_t> vac[2];      // per node
  std::vector<double> cen[2];       // per node, [N][3]
  std::vector<int32_t> vac_leaf[2]; // per neuron id (copy of the refresh input)
  bool counted = false;
};

namespace {

uint64_t quantise_axis(double x, double x0, double L) {
  double f = std::floor(((x - x0) / L) * kCells);
  if (!(f >= 0.0)) f = 0.0;                       // also maps -0.0
  if (f > kCells - 1.0) f = kCells - 1.0;
  return (uint64_t)f;
}

// Octant digit at depth k (1..21) is 4*bit(qx, 21-k) + 2*bit(qy, 21-k) + bit(qz, 21-k).
uint64_t morton_key(uint64_t qx, uint64_t qy, uint64_t qz) {
  uint64_t key = 0;
  for (int k = 1; k <= kMaxDepth; ++k) {
    int b = kMaxDepth - k;
    uint64_t digit = (((qx >> b) & 1) << 2) | (((qy >> b) & 1) << 1) | ((qz >> b) & 1);
    key = (key << 3) | digit;
  }
  return key;
}

uint64_t digit_at(uint64_t key, int k) {   // k in 1..21
  return (key >> (3 * (kMaxDepth - k))) & 7;
}

// Recursive subdivision: a node of depth k over sorted range [b, e) is inner iff it
// holds at least two neurons and k < 21; its children are the non-empty octants.
int64_t build_node(OracleTree& t, int depth, int64_t b, int64_t e) {
  int64_t idx = (int64_t)t.nodes.size();
  t.nodes.push_back(OracleNode());
  {
    OracleNode& nd = t.nodes[idx];
    nd.depth = depth;
    nd.prefix = depth == 0 ? 0 : (t.key[t.order[b]] >> (3 * (kMaxDepth - depth)));
    nd.begin = b;
    nd.end = e;
    nd.leaf = !((e - b) >= 2 && depth < kMaxDepth);
  }
  if (!t.nodes[idx].leaf) {
    int64_t s = b;
    std::vector<int64_t> kids;
    for (uint64_t d = 0; d < 8; ++d) {
      int64_t f = s;
      while (f < e && digit_at(t.key[t.order[f]], depth + 1) == d) ++f;
      if (f > s) kids.push_back(build_node(t, depth + 1, s, f));
      s = f;
    }
    t.nodes[idx].children = kids;
  }
  t.nodes[idx].subtree_end = (int64_t)t.nodes.size();
  return idx;
}

bool node_contains_key(const OracleNode& nd, uint64_t key) {
  if (nd.depth == 0) return true;
  return (key >> (3 * (kMaxDepth - nd.depth))) == nd.prefix;
}

// Aggregation (bottom-up, recursive): leaf = neuron position and count; inner =
// sum of the children, position = weighted average of the children, accumulated
// left to right in octant order, one rounding per operation.
void aggregate(OracleTree& t, int type, int64_t idx, const std::vector<double>& pos) {
  OracleNode& nd = t.nodes[idx];
  double* c = &t.cen[type][3 * idx];
  if (nd.leaf) {
    if (nd.end - nd.begin == 1) {
      int64_t id = t.order[nd.begin];
      t.vac[type][idx] = t.vac_leaf[type][id];
      c[0] = pos[3 * id + 0];
      c[1] = pos[3 * id + 1];
      c[2] = pos[3 * id + 2];
      return;
    }
    // bucket of coincident quantised points: members in id order
    int64_t v = 0;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t p = nd.begin; p < nd.end; ++p) {
      int64_t id = t.order[p];
      int64_t vj = t.vac_leaf[type][id];
      v += vj;
      if (vj > 0) {
        sx = sx + (double)vj * pos[3 * id + 0];
        sy = sy + (double)vj * pos[3 * id + 1];
        sz = sz + (double)vj * pos[3 * id + 2];
      }
    }
    t.vac[type][idx] = v;
    if (v > 0) { c[0] = sx / (double)v; c[1] = sy / (double)v; c[2] = sz / (double)v; }
    else { c[0] = c[1] = c[2] = 0.0; }
    return;
  }
  int64_t v = 0;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int64_t ch : nd.children) {
    aggregate(t, type, ch, pos);
    int64_t vk = t.vac[type][ch];
    v += vk;
    if (vk > 0) {
      const double* cc = &t.cen[type][3 * ch];
      sx = sx + (double)vk * cc[0];
      sy = sy + (double)vk * cc[1];
      sz = sz + (double)vk * cc[2];
    }
  }
  t.vac[type][idx] = v;
  if (v > 0) { c[0] = sx / (double)v; c[1] = sy / (double)v; c[2] = sz / (double)v; }
  else { c[0] = c[1] = c[2] = 0.0; }
}

// One entry of an accepted list: a neuron (leaf member) or a cell (inner node).
struct Entry {
  bool neuron;
  int64_t id;       // neuron id or node index
  double w;         // kernel weight
};

struct SearchCounters {
  int64_t visits = 0;   // node records read
  int64_t opens = 0;    // nodes replaced by their children (start node included)
};

struct Geometry {        // what the acceptance decisions and the weights read
  const std::vector<double>* pos;       // neuron positions
  const std::vector<double>* cen;       // node centroids of the searched type
};

// Squared distance: dx^2 + dy^2 + dz^2 with the last two terms fused (one rounding
// each for dx^2, dy^2 + that, dz^2 + that).
double dist2(const double* a, const double* b) {
  double dx = a[0] - b[0];
  double dy = a[1] - b[1];
  double dz = a[2] - b[2];
  return std::fma(dz, dz, std::fma(dy, dy, dx * dx));
}

double kernel_weight(int64_t v, double d2, double sigma) {
  return (double)v * std::exp(-(d2 / (sigma * sigma)));
}

// Visit node idx during the expansion of a start node for source `src`.
// `acc` supplies the acceptance geometry and `wgt` the weight geometry; they are
// the same except in the frozen-set evaluation used for finite differences.
void visit(const OracleTree& t, int type, int64_t src, int64_t idx, double sigma, double theta,
           const Geometry& acc, const Geometry& wgt, std::vector<Entry>& list,
           SearchCounters& cnt) {
  const OracleNode& nd = t.nodes[idx];
  cnt.visits += 1;
  if (t.vac[type][idx] == 0) return;                          // no vacancy: skip
  const double* xs_acc = &(*acc.pos)[3 * src];
  const double* xs_w = &(*wgt.pos)[3 * src];
  if (nd.leaf) {                                              // leaves are always accepted
    for (int64_t p = nd.begin; p < nd.end; ++p) {
      int64_t id = t.order[p];
      if (id == src) continue;                                // no autapse
      int64_t vj = t.vac_leaf[type][id];
      if (vj == 0) continue;
      double d2 = dist2(xs_w, &(*wgt.pos)[3 * id]);
      list.push_back(Entry{true, id, kernel_weight(vj, d2, sigma)});
    }
    return;
  }
  bool open;
  if (node_contains_key(nd, t.key[src])) {
    open = true;                                              // own cell: always opened
  } else {
    double d2 = dist2(xs_acc, &(*acc.cen)[3 * idx]);
    double l = std::ldexp(t.L, -nd.depth);                    // cube edge L / 2^k (exact)
    open = !(l * l < (theta * theta) * d2);
  }
  if (!open) {
    double d2 = dist2(xs_w, &(*wgt.cen)[3 * idx]);
    list.push_back(Entry{false, idx, kernel_weight(t.vac[type][idx], d2, sigma)});
    return;
  }
  cnt.opens += 1;
  for (int64_t ch : nd.children) visit(t, type, src, ch, sigma, theta, acc, wgt, list, cnt);
}

// The accepted list for a start node S: S itself is always opened.
void expand(const OracleTree& t, int type, int64_t src, int64_t S, double sigma, double theta,
            const Geometry& acc, const Geometry& wgt, std::vector<Entry>& list,
            SearchCounters& cnt) {
  list.clear();
  const OracleNode& nd = t.nodes[S];
  cnt.visits += 1;
  if (nd.leaf) {
    // only reachable for a one-node tree (the root is a leaf): list its members
    if (t.vac[type][S] == 0) return;
    for (int64_t p = nd.begin; p < nd.end; ++p) {
      int64_t id = t.order[p];
      if (id == src) continue;
      int64_t vj = t.vac_leaf[type][id];
      if (vj == 0) continue;
      double d2 = dist2(&(*wgt.pos)[3 * src], &(*wgt.pos)[3 * id]);
      list.push_back(Entry{true, id, kernel_weight(vj, d2, sigma)});
    }
    return;
  }
  cnt.opens += 1;
  for (int64_t ch : nd.children) visit(t, type, src, ch, sigma, theta, acc, wgt, list, cnt);
}

struct SearchResult {
  int64_t target = -1;
  double z0 = 0.0;          // normaliser of the level-0 list
  double window = 1.0;      // min over levels of |u - P/Z| at the chosen entry's bounds
  int32_t levels = 0;       // number of lists drawn from
  int64_t entries0 = 0;     // length of the level-0 list (its kernel evaluations)
  SearchCounters cnt;
};

SearchResult search_one(const OracleTree& t, int type, int64_t i, int64_t j, double sigma,
                        double theta, uint64_t seed, uint64_t step) {
  SearchResult res;
  Geometry g{&t.pos, &t.cen[type]};
  std::vector<Entry> list;
  int64_t S = 0;
  for (uint64_t level = 0;; ++level) {
    expand(t, type, i, S, sigma, theta, g, g, list, res.cnt);
    double Z = 0.0;
    for (const Entry& e : list) Z = Z + e.w;
    if (level == 0) {
      res.z0 = Z;
      res.entries0 = (int64_t)list.size();
    }
    res.levels += 1;
    if (list.empty() || Z == 0.0) { res.target = -1; return res; }
    double u = draw_u(seed, 0, (uint64_t)i, (uint64_t)j, step, level);
    double T = u * Z;
    int64_t chosen = -1;
    double P = 0.0, Pprev = 0.0;
    for (size_t e = 0; e < list.size(); ++e) {
      Pprev = P;
      P = P + list[e].w;
      if (P > T) { chosen = (int64_t)e; break; }
    }
    if (chosen < 0) {                                         // rounding: last positive entry
      for (size_t e = list.size(); e-- > 0;)
        if (list[e].w > 0.0) { chosen = (int64_t)e; break; }
      Pprev = P = Z;
    }
    double wd = std::min(std::fabs(u - Pprev / Z), std::fabs(P / Z - u));
    if (wd < res.window) res.window = wd;
    const Entry& ch = list[chosen];
    if (ch.neuron) { res.target = ch.id; return res; }
    S = ch.id;                                                // restart at the chosen cell
  }
}

}  // namespace

extern "C" {

// Build the octree over n neurons with positions pos[n][3] in the cube
// [box_min, box_min + box_edge)^3. Returns nullptr on invalid input.
OracleTree* oracle_build(const double* pos, int64_t n, const double* box_min, double box_edge) {
  if (n <= 0 || !(box_edge > 0.0) || !std::isfinite(box_edge)) return nullptr;
  for (int a = 0; a < 3; ++a) if (!std::isfinite(box_min[a])) return nullptr;
  for (int64_t i = 0; i < 3 * n; ++i) if (!std::isfinite(pos[i])) return nullptr;
  OracleTree* t = new OracleTree();
  t->n = n;
  t->L = box_edge;
  for (int a = 0; a < 3; ++a) t->x0[a] = box_min[a];
  t->pos.assign(pos, pos + 3 * n);
  t->key.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) q[a] = quantise_axis(pos[3 * i + a], t->x0[a], t->L);
    t->key[i] = morton_key(q[0], q[1], q[2]);
  }
  t->order.resize(n);
  for (int64_t i = 0; i < n; ++i) t->order[i] = i;
  std::sort(t->order.begin(), t->order.end(), [&](int64_t a, int64_t b) {
    if (t->key[a] != t->key[b]) return t->key[a] < t->key[b];
    return a < b;
  });
  build_node(*t, 0, 0, n);
  for (int ty = 0; ty < 2; ++ty) {
    t->vac[ty].assign(t->nodes.size(), 0);
    t->cen[ty].assign(3 * t->nodes.size(), 0.0);
  }
  return t;
}

void oracle_free(OracleTree* t) { delete t; }

int64_t oracle_num_nodes(const OracleTree* t) { return (int64_t)t->nodes.size(); }

void oracle_get_order(const OracleTree* t, int64_t* order, uint64_t* keys_by_id) {
  for (int64_t i = 0; i < t->n; ++i) { order[i] = t->order[i]; keys_by_id[i] = t->key[i]; }
}

// Topology in pre-order: depth, sorted-range [begin, end), pre-order subtree end, leaf flag.
void oracle_get_nodes(const OracleTree* t, int32_t* depth, int64_t* begin, int64_t* end,
                      int64_t* subtree_end, uint8_t* is_leaf) {
  for (size_t k = 0; k < t->nodes.size(); ++k) {
    const OracleNode& nd = t->nodes[k];
    depth[k] = nd.depth;
    begin[k] = nd.begin;
    end[k] = nd.end;
    subtree_end[k] = nd.subtree_end;
    is_leaf[k] = nd.leaf ? 1 : 0;
  }
}

// Refresh the per-type vacancy aggregates. Returns -1 if a count is negative.
int oracle_update_counts(OracleTree* t, const int32_t* vac_exc, const int32_t* vac_inh) {
  for (int64_t i = 0; i < t->n; ++i) if (vac_exc[i] < 0 || vac_inh[i] < 0) return -1;
  t->vac_leaf[0].assign(vac_exc, vac_exc + t->n);
  t->vac_leaf[1].assign(vac_inh, vac_inh + t->n);
  for (int ty = 0; ty < 2; ++ty) aggregate(*t, ty, 0, t->pos);
  t->counted = true;
  return 0;
}

void oracle_get_aggregates(const OracleTree* t, int type, int64_t* v, double* c) {
  size_t N = t->nodes.size();
  for (size_t k = 0; k < N; ++k) {
    v[k] = t->vac[type][k];
    c[3 * k + 0] = t->cen[type][3 * k + 0];
    c[3 * k + 1] = t->cen[type][3 * k + 1];
    c[3 * k + 2] = t->cen[type][3 * k + 2];
  }
}

// Run the searches (src[q], elem[q]) for q < n_sel. neuron_type selects the
// dendrite type searched (0 = excitatory, 1 = inhibitory).
// Outputs per search: target id or -1, level-0 normaliser, window distance, number
// of levels, node records read and nodes opened, and the length of the level-0 list.
int oracle_find_targets(const OracleTree* t, const uint8_t* neuron_type, double sigma,
                        double theta, uint64_t seed, uint64_t step, const int64_t* src,
                        const int64_t* elem, int64_t n_sel, int64_t* target, double* z0,
                        double* window, int32_t* levels, int64_t* visits, int64_t* opens,
                        int64_t* entries0, int nthreads) {
  if (!t->counted || !(sigma > 0.0) || !(theta >= 0.0)) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int64_t q = 0; q < n_sel; ++q) {
    int type = neuron_type[src[q]] ? 1 : 0;
    SearchResult r = search_one(*t, type, src[q], elem[q], sigma, theta, seed, step);
    target[q] = r.target;
    if (z0) z0[q] = r.z0;
    if (window) window[q] = r.window;
    if (levels) levels[q] = r.levels;
    if (visits) visits[q] = r.cnt.visits;
    if (opens) opens[q] = r.cnt.opens;
    if (entries0) entries0[q] = r.entries0;
  }
  return 0;
}

// Commit: group the requests with a target by (target, type), accept the
// min(requests, vacant) of highest priority (Philox stream 1, ties by (i, j)),
// emit the synapses sorted by (i, j), update the counts.
// elem_offset[n+1] is the CSR of searches by source; target[S].
// Synapse outputs must hold S entries; accepted_out[S] (may be null) receives the
// per-request accept flag. Returns the number formed.
int64_t oracle_commit(int64_t n, const int64_t* elem_offset, const int64_t* target,
                      const uint8_t* neuron_type, int32_t* vac_axon, int32_t* vac_exc,
                      int32_t* vac_inh, uint64_t seed, uint64_t step, int64_t* syn_src,
                      int64_t* syn_tgt, uint8_t* syn_type, uint8_t* accepted_out) {
  struct Req { int64_t g; int ty; uint64_t prio; int64_t i, j, s; };
  std::vector<Req> reqs;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t s = elem_offset[i]; s < elem_offset[i + 1]; ++s) {
      if (target[s] < 0) continue;
      int64_t j = s - elem_offset[i];
      P4 ctr = {{(uint64_t)i, (uint64_t)j, step, 0}};
      uint64_t prio = philox4x64_10(ctr, seed, 1).v[0];
      reqs.push_back(Req{target[s], neuron_type[i] ? 1 : 0, prio, i, j, s});
    }
  }
  std::sort(reqs.begin(), reqs.end(), [](const Req& a, const Req& b) {
    if (a.g != b.g) return a.g < b.g;
    if (a.ty != b.ty) return a.ty < b.ty;
    if (a.prio != b.prio) return a.prio < b.prio;
    if (a.i != b.i) return a.i < b.i;
    return a.j < b.j;
  });
  std::vector<uint8_t> accepted(elem_offset[n], 0);
  size_t a = 0;
  while (a < reqs.size()) {
    size_t b = a;
    while (b < reqs.size() && reqs[b].g == reqs[a].g && reqs[b].ty == reqs[a].ty) ++b;
    int64_t vac = reqs[a].ty ? vac_inh[reqs[a].g] : vac_exc[reqs[a].g];
    int64_t take = std::min<int64_t>((int64_t)(b - a), vac);
    for (int64_t k = 0; k < take; ++k) accepted[reqs[a + k].s] = 1;
    a = b;
  }
  int64_t formed = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t s = elem_offset[i]; s < elem_offset[i + 1]; ++s) {
      if (!accepted[s]) continue;
      int64_t g = target[s];
      int ty = neuron_type[i] ? 1 : 0;
      syn_src[formed] = i;
      syn_tgt[formed] = g;
      syn_type[formed] = (uint8_t)ty;
      ++formed;
      vac_axon[i] -= 1;
      if (ty) vac_inh[g] -= 1; else vac_exc[g] -= 1;
    }
  }
  if (accepted_out)
    for (int64_t s = 0; s < elem_offset[n]; ++s) accepted_out[s] = accepted[s];
  return formed;
}

// Philox4x64-10 block, exported for the pin against numpy.
void oracle_philox4x64_10(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
  P4 c = {{ctr[0], ctr[1], ctr[2], ctr[3]}};
  P4 r = philox4x64_10(c, key[0], key[1]);
  for (int k = 0; k < 4; ++k) out[k] = r.v[k];
}

// ---------------------------------------------------------------------------
// Expected attraction (differentiated form). For each source i with a_i > 0:
// Z_i = the level-0 normaliser; L = sum_i log Z_i. Gradients with the accepted
// sets held fixed: dZ_i/dx_i = sum_e w_e * (-2 (x_i - c_e) / sigma^2);
// dZ_i/dc_e = w_e * 2 (x_i - c_e) / sigma^2; a centroid is the vacancy-weighted mean
// of the neurons of its cell, so dc_C/dx_j = (v_j / v_C) I;
// dZ_i/dsigma = sum_e w_e * 2 d_e^2 / sigma^3.
// ---------------------------------------------------------------------------
namespace {

struct AttractionPass {
  std::vector<double> Z;
  double L = 0.0;
};

// Sum log Z_i with acceptance from `acc` and weights from `wgt`.
double attraction_sum(const OracleTree& t, const uint8_t* neuron_type, const int32_t* vac_axon,
                      double sigma, double theta, const Geometry acc[2], const Geometry wgt[2],
                      double* Z_out, int nthreads) {
  std::vector<double> logz(t.n, 0.0);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int64_t i = 0; i < t.n; ++i) {
    if (vac_axon[i] <= 0) { if (Z_out) Z_out[i] = 0.0; continue; }
    int ty = neuron_type[i] ? 1 : 0;
    std::vector<Entry> list;
    SearchCounters cnt;
    expand(t, ty, i, 0, sigma, theta, acc[ty], wgt[ty], list, cnt);
    double Z = 0.0;
    for (const Entry& e : list) Z = Z + e.w;
    if (Z_out) Z_out[i] = Z;
    if (Z > 0.0) logz[i] = std::log(Z);
  }
  double L = 0.0;                                  // serial sum: deterministic
  for (int64_t i = 0; i < t.n; ++i) L = L + logz[i];
  return L;
}

}  // namespace

// Z[n], L (scalar), dX[n][3], dsigma (scalar) at the tree's own geometry.
int oracle_attraction(const OracleTree* t, const uint8_t* neuron_type, const int32_t* vac_axon,
                      double sigma, double theta, double* Z, double* L, double* dX,
                      double* dsigma, int nthreads) {
  if (!t->counted || !(sigma > 0.0) || !(theta >= 0.0)) return -1;
  const int64_t n = t->n;
  const size_t N = t->nodes.size();
  Geometry g[2] = {{&t->pos, &t->cen[0]}, {&t->pos, &t->cen[1]}};
  *L = attraction_sum(*t, neuron_type, vac_axon, sigma, theta, g, g, Z, nthreads);
  // per-node gradient with respect to the centroid, per type
  std::vector<double> G[2] = {std::vector<double>(3 * N, 0.0), std::vector<double>(3 * N, 0.0)};
  std::vector<double> dx(3 * n, 0.0);
  double ds = 0.0;
  const double s2 = sigma * sigma, s3 = sigma * sigma * sigma;
  for (int64_t i = 0; i < n; ++i) {
    if (vac_axon[i] <= 0 || !(Z[i] > 0.0)) continue;
    int ty = neuron_type[i] ? 1 : 0;
    std::vector<Entry> list;
    SearchCounters cnt;
    expand(*t, ty, i, 0, sigma, theta, g[ty], g[ty], list, cnt);
    const double* xi = &t->pos[3 * i];
    for (const Entry& e : list) {
      const double* c = e.neuron ? &t->pos[3 * e.id] : &t->cen[ty][3 * e.id];
      double diff[3] = {xi[0] - c[0], xi[1] - c[1], xi[2] - c[2]};
      double d2 = dist2(xi, c);
      double f = e.w / Z[i];
      for (int a = 0; a < 3; ++a) {
        double gi = f * (-2.0 * diff[a] / s2);
        dx[3 * i + a] += gi;                       // through the source position
        if (e.neuron) dx[3 * e.id + a] -= gi;      // through a neuron target position
        else G[ty][3 * e.id + a] -= gi;            // through a cell centroid
      }
      ds += f * 2.0 * d2 / s3;
    }
  }
  // push the centroid gradients to the neurons of each cell: dc_C/dx_j = v_j / v_C
  for (int ty = 0; ty < 2; ++ty) {
    for (size_t k = 0; k < N; ++k) {
      const double* gk = &G[ty][3 * k];
      if (gk[0] == 0.0 && gk[1] == 0.0 && gk[2] == 0.0) continue;
      const OracleNode& nd = t->nodes[k];
      double vC = (double)t->vac[ty][k];
      for (int64_t p = nd.begin; p < nd.end; ++p) {
        int64_t id = t->order[p];
        double vj = (double)t->vac_leaf[ty][id];
        if (vj == 0.0) continue;
        for (int a = 0; a < 3; ++a) dx[3 * id + a] += gk[a] * (vj / vC);
      }
    }
  }
  for (int64_t k = 0; k < 3 * n; ++k) dX[k] = dx[k];
  *dsigma = ds;
  return 0;
}

// L at positions pos_new and width sigma_new, with the topology, the memberships
// and every acceptance decision taken at the tree's own geometry (frozen sets).
// Z_out[n] (nullable) receives every Z_i.
double oracle_attraction_frozen(const OracleTree* t, const uint8_t* neuron_type,
                                const int32_t* vac_axon, double sigma_new, double theta,
                                const double* pos_new, double* Z_out, int nthreads) {
  OracleTree moved = *t;                           // same topology and counts
  moved.pos.assign(pos_new, pos_new + 3 * t->n);
  for (int ty = 0; ty < 2; ++ty) aggregate(moved, ty, 0, moved.pos);
  Geometry acc[2] = {{&t->pos, &t->cen[0]}, {&t->pos, &t->cen[1]}};
  Geometry wgt[2] = {{&moved.pos, &moved.cen[0]}, {&moved.pos, &moved.cen[1]}};
  return attraction_sum(moved, neuron_type, vac_axon, sigma_new, theta, acc, wgt, Z_out,
                        nthreads);
}

// ---------------------------------------------------------------------------
// The change of the network between two connectivity updates (Sec. III-A, "Update of
// synaptic elements" and the first sub-phase of "Update of synapses"), as the
// multi-update workload reads it:
//   * calcium per neuron j and element kind k (0 axon, 1 excitatory dendrite,
//     2 inhibitory dendrite) is drawn from N(mean, sd): Box-Muller on Philox words
//     0 and 1 with key (seed, 2) and counter (j, k, step, 0);
//   * growth over the update: dz = steps * nu * (2 exp(-((Ca - xi) / zeta)^2) - 1),
//     xi = (eta + eps) / 2, zeta = (eps - eta) / (2 sqrt(ln 2)), so dz = 0 at
//     Ca = eta and at Ca = eps and dz = steps * nu at Ca = xi; z = max(z + dz, 0);
//   * round(frac * m) synapses are deleted uniformly at random: those of smallest
//     (Philox word 0, key (seed, 3), counter (s, step, 0, 0); then s), s being the
//     synapse's place in the list at the start of the step;
//   * then for k = 0, 1, 2 in turn: where floor(z) fell below the bound elements of
//     kind k, that many of the neuron's synapses of that kind break, those of smallest
//     (top 32 bits of Philox word 0, key (seed, 4), counter (s, step, k, 0); then s).
//     A synapse (i, g, type) binds one axonal element of i and one dendritic element
//     of kind 1 + type of g; breaking it frees both.
//   * the list keeps its order; vacant elements are floor(z) - bound.
// ---------------------------------------------------------------------------
double oracle_growth_delta(double ca, double nu, double eps, double eta, int32_t steps) {
  const double xi = 0.5 * (eta + eps);
  const double zeta = (eps - eta) / (2.0 * std::sqrt(std::log(2.0)));
  const double r = (ca - xi) / zeta;
  const double e = std::exp(-(r * r));
  return (double)steps * nu * (2.0 * e - 1.0);
}

double oracle_calcium(uint64_t seed, uint64_t j, uint64_t k, uint64_t step, double mean,
                      double sd) {
  P4 ctr = {{j, k, step, 0}};
  P4 w = philox4x64_10(ctr, seed, 2);
  const double u1 = (double)((w.v[0] >> 11) + 1) * 0x1p-53;     // (0, 1]
  const double u2 = (double)(w.v[1] >> 11) * 0x1p-53;           // [0, 1)
  const double two_pi = 6.283185307179586476925286766559;
  const double g = std::sqrt(-2.0 * std::log(u1)) * std::cos(two_pi * u2);
  return mean + sd * g;
}

// Appends m_new synapses at [m, m + m_new) and binds their elements.
void oracle_plasticity_record(int64_t n, int64_t m, int64_t m_new, const int32_t* nsrc,
                              const int32_t* ntgt, const uint8_t* ntype, int32_t* src,
                              int32_t* tgt, uint8_t* type, int32_t* bound) {
  for (int64_t q = 0; q < m_new; ++q) {
    src[m + q] = nsrc[q];
    tgt[m + q] = ntgt[q];
    type[m + q] = ntype[q];
    bound[nsrc[q]] += 1;
    bound[(1 + (int64_t)ntype[q]) * n + ntgt[q]] += 1;
  }
}

// One step; z [3][n], bound [3][n] and the list (m entries) are updated in place,
// vac [3][n] receives the vacant elements. Returns the new list length.
int64_t oracle_plasticity_step(int64_t n, int64_t m, double nu, double eps, double eta,
                               int32_t steps, double ca_mean, double ca_sd, double delete_frac,
                               uint64_t seed, uint64_t step, double* z, int32_t* bound,
                               int32_t* src, int32_t* tgt, uint8_t* type, int32_t* vac) {
  for (int64_t k = 0; k < 3; ++k)
    for (int64_t j = 0; j < n; ++j) {
      const double ca = oracle_calcium(seed, (uint64_t)j, (uint64_t)k, step, ca_mean, ca_sd);
      const double zz = z[k * n + j] + oracle_growth_delta(ca, nu, eps, eta, steps);
      z[k * n + j] = zz > 0.0 ? zz : 0.0;
    }
  std::vector<char> dead(m, 0);
  auto unbind = [&](int64_t s) {
    dead[s] = 1;
    bound[src[s]] -= 1;
    bound[(1 + (int64_t)type[s]) * n + tgt[s]] -= 1;
  };
  // deletion
  const int64_t n_del = (int64_t)std::floor(delete_frac * (double)m + 0.5);
  {
    std::vector<std::pair<uint64_t, int64_t>> pr(m);
    for (int64_t s = 0; s < m; ++s) {
      P4 ctr = {{(uint64_t)s, step, 0, 0}};
      pr[s] = {philox4x64_10(ctr, seed, 3).v[0], s};
    }
    std::sort(pr.begin(), pr.end());
    for (int64_t q = 0; q < n_del && q < m; ++q) unbind(pr[q].second);
  }
  // retraction, kind by kind
  for (int k = 0; k < 3; ++k) {
    std::vector<int64_t> excess(n);
    for (int64_t j = 0; j < n; ++j)
      excess[j] = (int64_t)bound[k * n + j] - (int64_t)std::floor(z[k * n + j]);
    struct C { int64_t owner; uint32_t q; int64_t s; };
    std::vector<C> cand;
    for (int64_t s = 0; s < m; ++s) {
      if (dead[s]) continue;
      int64_t owner;
      if (k == 0) owner = src[s];
      else if ((int)type[s] == k - 1) owner = tgt[s];
      else continue;
      if (excess[owner] <= 0) continue;
      P4 ctr = {{(uint64_t)s, step, (uint64_t)k, 0}};
      cand.push_back({owner, (uint32_t)(philox4x64_10(ctr, seed, 4).v[0] >> 32), s});
    }
    std::sort(cand.begin(), cand.end(), [](const C& a, const C& b) {
      if (a.owner != b.owner) return a.owner < b.owner;
      if (a.q != b.q) return a.q < b.q;
      return a.s < b.s;
    });
    for (size_t p = 0; p < cand.size();) {
      size_t e = p;
      while (e < cand.size() && cand[e].owner == cand[p].owner) ++e;
      const int64_t drop = std::min<int64_t>(excess[cand[p].owner], (int64_t)(e - p));
      for (int64_t q = 0; q < drop; ++q) unbind(cand[p + q].s);
      p = e;
    }
  }
  int64_t w = 0;
  for (int64_t s = 0; s < m; ++s) {
    if (dead[s]) continue;
    src[w] = src[s];
    tgt[w] = tgt[s];
    type[w] = type[s];
    ++w;
  }
  for (int64_t k = 0; k < 3; ++k)
    for (int64_t j = 0; j < n; ++j)
      vac[k * n + j] = (int32_t)((int64_t)std::floor(z[k * n + j]) - bound[k * n + j]);
  return w;
}


// ---------------------------------------------------------------------------
// Electrical activity between connectivity updates (Sec. II, "Update of electrical
// activity") with the firing-rate approximation of Sec. IV-B. One step is 1 ms:
//   1. exchange: the spikes a neuron recorded in the previous step reach its synapse
//      partners. Under the approximation, a synapse whose two neurons lie in
//      different processes (approx = 1; every synapse with approx = 2) carries a
//      spike at step t iff u < f_i, f_i being the source's firing frequency over the
//      previous epoch (spikes per step) and u = (Philox word 0 >> 11) * 2^-53 with
//      key (seed, 5) and counter (synapse s, t, 0, 0). Per target g: e_g excitatory
//      and h_g inhibitory spikes received (the synapse type is the source's type);
//   2. neuron model (Izhikevich 2003; regular spiking for excitatory, fast spiking
//      for inhibitory neurons): I = w_e e_g - w_i h_g + mu + width (u' - 1/2) with u'
//      from key (seed, 6), counter (g, t, 0, 0); v += (0.04 v^2 + 5 v + 140 - u + I)/2
//      twice (two half-millisecond steps), u += a (b v - u); v >= 30 is a spike:
//      v = c, u += d, and the spike is recorded for the next step;
//   3. calcium (a running average of the firing rate): Ca -= Ca / tau, then
//      Ca += beta for a spike;
//   4. every epoch (delta steps; the step t with (t + 1) % delta == 0 closes one) the
//      frequency f = spikes in the epoch / delta replaces the previous one.
// Every operation is a +, -, * or a comparison in fp64 (1/tau and 1/delta are
// passed in), so the library's result is the same bit for bit.
// last_input (nullable) [2][n] receives e and h of the last step.
// ---------------------------------------------------------------------------
int64_t oracle_activity_run(int64_t n, const uint8_t* ntype, const int32_t* rank,
                            int64_t m, const int32_t* src, const int32_t* tgt,
                            const uint8_t* stype, int32_t approx, const double* p,
                            double inv_tau, double inv_delta, int32_t delta, uint64_t seed,
                            uint64_t t0, int32_t steps, double* v, double* u, double* ca,
                            uint8_t* spk, int32_t* count, double* freq, int32_t* last_input) {
  // p: a_e b_e c_e d_e a_i b_i c_i d_i w_e w_i mu width beta
  std::vector<int32_t> e(n), h(n);
  std::vector<uint8_t> fired(n);
  int64_t total = 0;
  for (int32_t k = 0; k < steps; ++k) {
    const uint64_t t = t0 + (uint64_t)k;
    std::fill(e.begin(), e.end(), 0);
    std::fill(h.begin(), h.end(), 0);
    for (int64_t s = 0; s < m; ++s) {
      const int32_t i = src[s], g = tgt[s];
      const bool remote = approx == 2 || (approx == 1 && rank && rank[i] != rank[g]);
      bool arrives;
      if (remote) {
        P4 ctr = {{(uint64_t)s, t, 0, 0}};
        const double uu = (double)(philox4x64_10(ctr, seed, 5).v[0] >> 11) * 0x1p-53;
        arrives = uu < freq[i];
      } else {
        arrives = spk[i] != 0;
      }
      if (arrives) {
        if (stype[s] == 0) e[g] += 1; else h[g] += 1;
      }
    }
    for (int64_t g = 0; g < n; ++g) {
      const double* q = ntype[g] ? p + 4 : p;
      P4 ctr = {{(uint64_t)g, t, 0, 0}};
      const double uu = (double)(philox4x64_10(ctr, seed, 6).v[0] >> 11) * 0x1p-53;
      const double I = p[8] * (double)e[g] - p[9] * (double)h[g] + (p[10] + p[11] * (uu - 0.5));
      double vv = v[g], w = u[g];
      vv = vv + 0.5 * (0.04 * vv * vv + 5.0 * vv + 140.0 - w + I);
      vv = vv + 0.5 * (0.04 * vv * vv + 5.0 * vv + 140.0 - w + I);
      w = w + q[0] * (q[1] * vv - w);
      const bool f = vv >= 30.0;
      if (f) {
        vv = q[2];
        w = w + q[3];
      }
      v[g] = vv;
      u[g] = w;
      double c = ca[g];
      c = c - c * inv_tau;
      if (f) c = c + p[12];
      ca[g] = c;
      fired[g] = f ? 1 : 0;
      count[g] += f ? 1 : 0;
      total += f ? 1 : 0;
      if ((t + 1) % (uint64_t)delta == 0) {
        freq[g] = (double)count[g] * inv_delta;
        count[g] = 0;
      }
    }
    std::memcpy(spk, fired.data(), (size_t)n);
    if (last_input && k == steps - 1) {
      std::memcpy(last_input, e.data(), sizeof(int32_t) * n);
      std::memcpy(last_input + n, h.data(), sizeof(int32_t) * n);
    }
  }
  return total;
}

}  // extern "C"
