// Device-wide exclusive prefix sums and an LSD radix sort of (64-bit key, int32 value).
#pragma once

#include <algorithm>

#include "common.hpp"

namespace msp {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

// Exclusive scan of one value per thread across a 256-thread block (4 waves).
template <class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds4, T* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  T x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) lds4[w] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanBlock / kWave; ++k) {
    T s = lds4[k];
    off += (k < w) ? s : T(0);
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

// Scans take an optional device count dn (nullable): the items are then the first
// min(n, *dn) (a negative count is 0), the launches stay sized for n + 1 items and the
// total goes to out[count].
__device__ __forceinline__ int64_t scan_count(int64_t n, const int64_t* dn) {
  if (!dn) return n;
  const int64_t c = *dn;
  return c < 0 ? 0 : (c < n ? c : n);
}

template <class T, class Tin, class F>
__global__ void __launch_bounds__(kScanBlock) scan_reduce_k(const Tin* in, int64_t n, T* sums, F f,
                                                           const int64_t* dn) {
  __shared__ T lds4[kScanBlock / kWave];
  n = scan_count(n, dn);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= n) {                      // past a device count: an empty block
    if (threadIdx.x == 0) sums[blockIdx.x] = 0;
    return;
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t idx = base + (int64_t)k * kScanBlock + threadIdx.x;
    if (idx < n) s += f(in ? in[idx] : Tin(), idx);
  }
  T tot;
  (void)block_exclusive_scan<T>(s, lds4, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[i] = sum_{k<i} f(in[k]) + offsets[block]; if total_out, out[n] = grand total.
template <class T, class Tin, class F>
__global__ void __launch_bounds__(kScanBlock) scan_apply_k(const Tin* in, int64_t n, T* out,
                                                          const T* offsets, F f, int write_total,
                                                          const int64_t* dn) {
  __shared__ T lds4[kScanBlock / kWave];
  n = scan_count(n, dn);
  if ((int64_t)blockIdx.x * kScanTile > n) return;   // nothing to write (uniform)
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t idx = base + k;
    v[k] = idx < n ? f(in ? in[idx] : Tin(), idx) : T(0);
    s += v[k];
  }
  T tot;
  T pre = block_exclusive_scan<T>(s, lds4, &tot);
  pre += offsets ? offsets[blockIdx.x] : T(0);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t idx = base + k;
    if (idx < n || (dn && write_total && idx == n)) out[idx] = pre;
    pre += v[k];
  }
  if (!dn && write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanBlock - 1)
    out[n] = pre;
}

template <class T>
__global__ void fill_scalar_k(T* p, T v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

template <class T>
struct Ident {
  __device__ T operator()(T x, int64_t) const { return x; }
};

// Bytes of block-sum scratch an exclusive scan of n elements of T needs.
template <class T>
size_t scan_tmp_bytes(int64_t n) {
  size_t bytes = 0;
  while (n > kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    bytes += (sizeof(T) * (size_t)n + 255) & ~(size_t)255;
  }
  return bytes + 256;
}

// Exclusive scan of f(in[i], i) into out[0..n) (and out[n] = total if write_total).
// `in` may be null (f then sees a default value) and may alias `out` element for
// element. Block sums go to `tmp` (scan_tmp_bytes<T>(n) bytes) or, if null, to
// stream-ordered temporary memory. With a device count dn (see scan_count) the scan
// covers its first min(n, *dn) items, writes the total after them, and needs
// scan_tmp_bytes<T>(n + 1) bytes of `tmp`.
template <class T, class Tin, class F>
hipError_t exclusive_scan(const Tin* in, T* out, int64_t n, F f, bool write_total, hipStream_t s,
                          void* tmp = nullptr, const int64_t* dn = nullptr) {
  if (n <= 0) {
    if (write_total) {
      fill_scalar_k<T><<<1, 64, 0, s>>>(out, T(0));
      return hipGetLastError();
    }
    return hipSuccess;
  }
  // with a device count the launch also covers position n, where the total may go
  const int64_t nb = (n + (dn ? 1 : 0) + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    scan_apply_k<T, Tin, F><<<1, kScanBlock, 0, s>>>(in, n, out, nullptr, f, write_total ? 1 : 0,
                                                     dn);
    return hipGetLastError();
  }
  Temp own(s);
  T* sums;
  void* rest = nullptr;
  if (tmp) {
    sums = static_cast<T*>(tmp);
    rest = static_cast<char*>(tmp) + ((sizeof(T) * (size_t)nb + 255) & ~(size_t)255);
  } else {
    hipError_t e = own.alloc(sizeof(T) * (size_t)nb);
    if (e != hipSuccess) return e;
    sums = own.as<T>();
  }
  scan_reduce_k<T, Tin, F><<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, sums, f, dn);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = exclusive_scan<T, T, Ident<T>>(sums, sums, nb, Ident<T>(), false, s, rest);
  if (e != hipSuccess) return e;
  scan_apply_k<T, Tin, F><<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, out, sums, f,
                                                             write_total ? 1 : 0, dn);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LSD radix sort, 8-bit digits. Stable: equal keys keep their input order, so
// sorting (key, id) pairs that start in id order yields (key, id) order.
// ---------------------------------------------------------------------------
constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int64_t kSortGridDn = 1024;   // blocks of a device-counted sort's passes

// dn (nullable): a device count that lowers n (items past it are left alone; the
// tiles beyond it contribute empty histograms and write nothing).
__device__ __forceinline__ int64_t sort_count(int64_t n, const int32_t* dn) {
  if (!dn) return n;
  const int64_t c = *dn;
  return c < 0 ? 0 : (c < n ? c : n);
}

// With a device count the histograms cover only the tiles that hold items: nbd (device)
// is their number, and it replaces nb in the digit-major layout. A block takes tiles
// blockIdx.x, + gridDim.x, ... (a device-counted sort launches fewer blocks than tiles).
__global__ void __launch_bounds__(kSortBlock) rs_hist_k(const uint64_t* keys, int64_t n, int shift,
                                                       uint32_t* hist, int nb, const int32_t* dn,
                                                       const int32_t* nbd) {
  if (nbd) nb = *nbd;
  __shared__ uint32_t h[256];
  n = sort_count(n, dn);
  for (int tile = blockIdx.x; tile < nb; tile += gridDim.x) {   // uniform over the block
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)tile * kSortTile;
    for (int k = 0; k < kSortItems && base < n; ++k) {
      int64_t idx = base + (int64_t)k * kSortBlock + threadIdx.x;
      if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + tile] = h[threadIdx.x];
    __syncthreads();                    // h is cleared for the next tile
  }
}

// One tile of kSortTile items: ranked by digit (stable) into LDS first, then written
// out digit run by digit run, so consecutive threads store to consecutive addresses.
// The tile's count of each digit is the difference of consecutive entries of the
// scanned (digit-major) histogram.
__global__ void __launch_bounds__(kSortBlock) rs_scatter_k(const uint64_t* kin, const int32_t* vin,
                                                          uint64_t* kout, int32_t* vout, int64_t n,
                                                          int shift, const uint32_t* off, int nb,
                                                          const int32_t* dn, const int32_t* nbd) {
  if (nbd) nb = *nbd;
  __shared__ uint64_t lk[kSortTile];
  __shared__ int32_t lv[kSortTile];
  __shared__ uint32_t lstart[256];      // tile-local start of each digit's run
  __shared__ uint32_t gstart[256];      // global start of this tile's run of each digit
  __shared__ uint32_t run[256];         // items of each digit placed so far
  __shared__ uint32_t wcnt[kSortBlock / kWave][256];
  const int t = threadIdx.x;
  const int w = t / kWave;
  const int lane = t & (kWave - 1);
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (kWave - lane));
  n = sort_count(n, dn);
  for (int tile = blockIdx.x; tile < nb; tile += gridDim.x) {   // uniform over the block
    const int64_t base = (int64_t)tile * kSortTile;
    if (base >= n) break;
    const int64_t rem = n - base;
    const int tile_n = rem < kSortTile ? (int)rem : kSortTile;
    const int64_t h = (int64_t)t * nb + tile;
    const uint32_t g0 = off[h];
    const uint32_t g1 = h + 1 < 256 * (int64_t)nb ? off[h + 1] : (uint32_t)n;
    const uint32_t count = g1 - g0;     // this tile's items of digit t
    gstart[t] = g0;
    lstart[t] = count;
    run[t] = 0;
    __syncthreads();
    // inclusive scan of the 256 counts (Hillis-Steele), then exclusive = inclusive - own
    for (int d = 1; d < 256; d <<= 1) {
      const uint32_t v = t >= d ? lstart[t - d] : 0u;
      __syncthreads();
      lstart[t] += v;
      __syncthreads();
    }
    lstart[t] -= count;
    // the tile's items in registers first: one memory round trip per tile, not per round
    uint64_t keys[kSortItems];
    int32_t vals[kSortItems];
#pragma unroll
    for (int c = 0; c < kSortItems; ++c) {
      const int li = c * kSortBlock + t;
      keys[c] = li < tile_n ? kin[base + li] : 0ull;
      vals[c] = li < tile_n ? vin[base + li] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kSortItems; ++c) {
#pragma unroll
      for (int k = 0; k < kSortBlock / kWave; ++k) wcnt[k][t] = 0;
      __syncthreads();
      const int li = c * kSortBlock + t;
      const bool valid = li < tile_n;
      const uint64_t key = keys[c];
      const uint32_t d = (uint32_t)(key >> shift) & 255u;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        peers &= bit ? bb : ~bb;
      }
      const uint32_t rank = (uint32_t)__popcll(peers & lt);
      if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
      __syncthreads();
      if (valid) {
        uint32_t p = lstart[d] + run[d] + rank;
        for (int k = 0; k < w; ++k) p += wcnt[k][d];
        if (p < (uint32_t)kSortTile) {
          lk[p] = key;
          lv[p] = vals[c];
        }
      }
      __syncthreads();
      uint32_t add = 0;
#pragma unroll
      for (int k = 0; k < kSortBlock / kWave; ++k) add += wcnt[k][t];
      run[t] += add;
    }
    __syncthreads();
    for (int i = t; i < tile_n; i += kSortBlock) {
      const uint64_t key = lk[i];
      const uint32_t d = (uint32_t)(key >> shift) & 255u;
      const uint32_t g = gstart[d] + ((uint32_t)i - lstart[d]);
      if ((int64_t)g < n) {
        kout[g] = key;
        vout[g] = lv[i];
      }
    }
    __syncthreads();                    // the shared arrays are reused by the next tile
  }
}

__global__ void __launch_bounds__(kSortBlock) rs_copy_k(const uint64_t* __restrict__ kin,
                                                       const int32_t* __restrict__ vin,
                                                       uint64_t* __restrict__ kout,
                                                       int32_t* __restrict__ vout, int64_t n,
                                                       const int32_t* dn) {
  const int64_t c = sort_count(n, dn);
  for (int64_t i = gtid(); i < c; i += gstride()) {
    kout[i] = kin[i];
    vout[i] = vin[i];
  }
}

// The tiles that hold the first min(n, *dn) items (as int32 for the kernels) and their
// histogram entries (as int64 for the scan).
__global__ void rs_tiles_k(int64_t n, const int32_t* dn, int32_t* nbd, int64_t* hn) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t c = sort_count(n, dn);
  const int64_t t = (c + kSortTile - 1) / kSortTile;
  *nbd = (int32_t)t;
  *hn = 256 * t;
}

// Scratch bytes of radix_sort_pairs_ws for n items: the digit histograms, the block
// sums of their scan, and the tile counts of a device-counted sort.
inline size_t radix_sort_ws_bytes(int64_t n) {
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  const size_t hist = ((sizeof(uint32_t) * 256 * (size_t)(nb > 0 ? nb : 1)) + 255) & ~(size_t)255;
  return hist + scan_tmp_bytes<uint32_t>(256 * (nb > 0 ? nb : 1) + 1) + 256;
}

// Sort (keys, vals) of length n ascending by the low `bits` key bits (a multiple of 8).
// Buffers k0/v0 hold the input and receive the output; k1/v1 are scratch of size n;
// `ws` holds radix_sort_ws_bytes(n) bytes. Allocates nothing, so it can be captured.
// dn (nullable, device): sort only the first min(n, *dn) items, a count known on the
// device alone; the launches stay sized for n.
inline hipError_t radix_sort_pairs_ws(uint64_t* k0, int32_t* v0, uint64_t* k1, int32_t* v1,
                                      int64_t n, int bits, hipStream_t s, void* ws,
                                      const int32_t* dn = nullptr) {
  if (n <= 1) return hipSuccess;
  const int64_t nb = (n + kSortTile - 1) / kSortTile;
  uint32_t* hist = static_cast<uint32_t*>(ws);
  const size_t hist_bytes = ((sizeof(uint32_t) * 256 * (size_t)nb) + 255) & ~(size_t)255;
  void* scan_ws = static_cast<char*>(ws) + hist_bytes;
  // a device-counted sort sizes its histograms by the tiles that hold items
  int32_t* nbd = nullptr;
  int64_t* hn = nullptr;
  if (dn) {
    char* tail = static_cast<char*>(scan_ws) + scan_tmp_bytes<uint32_t>(256 * nb + 1);
    hn = reinterpret_cast<int64_t*>(tail);
    nbd = reinterpret_cast<int32_t*>(tail + sizeof(int64_t));
    rs_tiles_k<<<1, 64, 0, s>>>(n, dn, nbd, hn);
  }
  uint64_t* ka = k0;
  int32_t* va = v0;
  uint64_t* kb = k1;
  int32_t* vb = v1;
  hipError_t e = hipSuccess;
  // a device-counted sort holds few tiles with items, mostly: a bounded grid loops
  const unsigned grid = dn ? (unsigned)std::min<int64_t>(nb, kSortGridDn) : (unsigned)nb;
  for (int shift = 0; shift < bits; shift += 8) {
    rs_hist_k<<<grid, kSortBlock, 0, s>>>(ka, n, shift, hist, (int)nb, dn, nbd);
    e = exclusive_scan<uint32_t, uint32_t, Ident<uint32_t>>(hist, hist, 256 * nb, Ident<uint32_t>(),
                                                            false, s, scan_ws, hn);
    if (e != hipSuccess) return e;
    rs_scatter_k<<<grid, kSortBlock, 0, s>>>(ka, va, kb, vb, n, shift, hist, (int)nb, dn, nbd);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t* tk = ka; ka = kb; kb = tk;
    int32_t* tv = va; va = vb; vb = tv;
  }
  if (ka != k0) {
    if (dn) {                           // an odd number of passes: copy the sorted items
      rs_copy_k<<<grid_cap(n, kSortBlock), kSortBlock, 0, s>>>(ka, va, k0, v0, n, dn);
      return hipGetLastError();
    }
    e = hipMemcpyAsync(k0, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(v0, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
  }
  return e;
}

// Sort (keys, vals) of length n ascending by key; `bits` = number of key bits to sort.
// Buffers k0/v0 hold the input and receive the output; k1/v1 are scratch of size n.
inline hipError_t radix_sort_pairs(uint64_t* k0, int32_t* v0, uint64_t* k1, int32_t* v1, int64_t n,
                                   int bits, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  Temp ws(s);
  hipError_t e = ws.alloc(radix_sort_ws_bytes(n));
  if (e != hipSuccess) return e;
  return radix_sort_pairs_ws(k0, v0, k1, v1, n, bits, s, ws.p);
}

}  // namespace msp
