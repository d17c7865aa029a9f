// Hash accumulator for wide outputs (Sec. III-C: past d = 1024 the dense
// accumulator no longer fits the nearest cache level and a hash table is used
// instead).
//
// Products are walked as one flat list per group of A entries: 64 A entries
// are staged at a time (their B row start, length and value), an inclusive
// scan of the lengths lets lane t find its product by a binary search over
// the staged prefix sums, so every lane has work however short the B rows
// are. Lanes issue the B loads of kGather products before using any.
//
// First, products per row (k_hash_flops) and their log2 histogram
// (k_hash_hist). Rows with at least the threshold hash_split_choose takes
// from it are split rows: power-law inputs have hubs whose product lists
// would keep one wavefront busy for the whole launch. The threshold is
// kHashSplitMin unless the rows above it would need more bitmap memory than
// the split budget; then it is the least power of two whose rows fit, so the
// longest rows are always split.
//
// Short rows (below the threshold), one wavefront each:
// - symbolic: the distinct columns (minus masked ones) are counted in an LDS
//   bitmap of d bits for d <= 32 kRankWords, else in an LDS open-addressing
//   set (linear probing, column as key) of a power of two >= 2 min(d,
//   flops_i) slots, or, when that exceeds the set, in the d-bit bitmap;
// - numeric: rows with at most kHashNumMax outputs accumulate in an LDS table
//   of (column, sum) slots sized from the exact output count, one launch per
//   table size class over that class's row list (k_hash_table_bins). The row
//   is put in column order by rank in an LDS bitmap of the row (d <= 32
//   kRankWords), or by compacting the occupied slots and sorting them
//   (bitonic, in LDS). Rows with more outputs (only rows left unsplit by a
//   forced slot bound) mark an LDS bitmap and add into a private d-wide strip
//   in global memory; the row is written by walking the bitmap and the strip
//   is cleared behind it.
//
// Split rows: chunks of split_chunk_entries A entries, one workgroup each. Symbolic
// chunks OR their columns into the row's global bitmap (an LDS copy first,
// then one atomic OR per non-zero word); a count pass gives the row's output
// count and, per bitmap word, the outputs before it. Numeric chunks add each
// product at its column's rank in that bitmap, into an LDS array of the
// row's outputs (then one global atomic add per output); an emit pass writes
// the row in column order. A row of one chunk is written by its chunk
// directly. A row with more outputs than that LDS array is cut into windows
// of output positions instead: a workgroup per window takes each A entry's
// products in the window's column range (binary search in the sorted B
// row) and writes the window. Wide rows reuse each column little, so global
// atomic adds would cost one per product.
//
// Slots, chunks, accumulators, windows and class lists are reserved per
// group of rows or slots with one global atomic add each: device-scope
// atomics that every row sends to one counter serialize.
//
// Masked columns are tested per product (binary search in the mask row, or a
// bit test), so tables and bitmaps only ever hold output columns.
#include <cstdlib>
#include <type_traits>

#include "api_internal.hpp"
#include "dev_numeric.hpp"

namespace tss {

constexpr uint32_t kEmpty = 0xffffffffu;  // empty slot; sorts after every column
constexpr int kSymSlots = 2048;           // LDS words per wavefront (8 KB): set slots or d-bit bitmap words
constexpr int kNumSlots = 1024;           // numeric table slots per wavefront (power of two)
constexpr int kHashNumMax = kNumSlots / 2;  // numeric rows up to this many outputs use the table
constexpr int kHashWaves = 4;             // wavefronts (rows) per workgroup
constexpr int kDenseFetch = 16;           // rows a dense-row worker takes per fetch
constexpr int kSplitWaves = 4;            // wavefronts per chunk workgroup
constexpr int kSplitEntries = kSplitWaves * kWave;  // A entries per symbolic chunk (a wavefront stages 64)
constexpr int kRankWords = 256;           // up to this many bitmap words (d <= 8192): narrow kernels
constexpr int kWinWaves = 4;              // wavefronts per output-window workgroup
constexpr int kSplitSmall = 1024;         // chunks of rows with at most this many outputs use a small LDS array
static_assert(kHashMaxD <= kSymSlots * 32, "the d-bit bitmap of a row must fit a wavefront's LDS words");

__device__ __forceinline__ uint32_t hslot(int32_t j, uint32_t mask) { return ((uint32_t)j * 2654435761u) & mask; }

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t x) {
  uint32_t p = 64;
  while (p < x) p <<= 1;
  return p;
}

__device__ __forceinline__ bool is_masked(const HashMask& m, int64_t row, int32_t j) {
  if (m.bits) return (m.bits[row * m.wpm + (j >> 5)] >> (j & 31)) & 1u;
  if (m.rp) {
    int lo = m.rp[row], hi = m.rp[row + 1];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const int32_t v = m.ci[mid];
      if (v == j) return true;
      if (v < j)
        lo = mid + 1;
      else
        hi = mid;
    }
  }
  return false;
}

// Stage A entries [base, base + nb) of a row (nb <= 64): lane t holds entry
// base + t's B row start and value, and pref[t + 1] the inclusive sum of the
// B row lengths (pref[0] = 0). Returns the number of products staged.
template <typename T>
__device__ __forceinline__ int stage_products(const Problem& pr, int base, int nb, int* start, int* pref, T* aval_s) {
  const int lane = threadIdx.x & (kWave - 1);
  int q0 = 0, len = 0;
  T a = T(0);
  if (lane < nb) {
    const int k = pr.aci[base + lane];
    q0 = pr.brp[k];
    len = pr.brp[k + 1] - q0;
    if constexpr (!std::is_same<T, char>::value) a = ((const T*)pr.aval)[base + lane];
  }
  int incl = len;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  wave_sync();
  start[lane] = q0;
  pref[lane + 1] = incl;
  if (lane == 0) pref[0] = 0;
  if constexpr (!std::is_same<T, char>::value) aval_s[lane] = a;
  wave_sync();
  return __shfl(incl, kWave - 1, kWave);
}

// As stage_products, but only the products of columns [c_lo, c_hi): lane t's
// B row is cut to that range by binary search (B rows are sorted). The
// first window needs no lower search and the last no upper one: products
// outside the row's output columns are masked ones, which the caller skips.
template <typename T>
__device__ __forceinline__ int stage_window(const Problem& pr, int base, int nb, int c_lo, int c_hi, bool first,
                                            bool last, int* start, int* pref, T* aval_s) {
  const int lane = threadIdx.x & (kWave - 1);
  int q0 = 0, len = 0;
  T a = T(0);
  if (lane < nb) {
    const int k = pr.aci[base + lane];
    // first entries >= c_lo and >= c_hi, the two searches side by side (two
    // loads in flight per step)
    int l0 = pr.brp[k], h0 = pr.brp[k + 1], l1 = l0, h1 = h0;
    if (first) h0 = l0;  // lower end: the row start
    if (last) l1 = h1;   // upper end: the row end
    while (l0 < h0 || l1 < h1) {
      const int m0 = (l0 + h0) >> 1, m1 = (l1 + h1) >> 1;
      const int v0 = l0 < h0 ? pr.bci[m0] : 0, v1 = l1 < h1 ? pr.bci[m1] : 0;
      if (l0 < h0) {
        if (v0 < c_lo)
          l0 = m0 + 1;
        else
          h0 = m0;
      }
      if (l1 < h1) {
        if (v1 < c_hi)
          l1 = m1 + 1;
        else
          h1 = m1;
      }
    }
    q0 = l0;
    len = l1 - l0;
    a = ((const T*)pr.aval)[base + lane];
  }
  int incl = len;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  wave_sync();
  start[lane] = q0;
  pref[lane + 1] = incl;
  if (lane == 0) pref[0] = 0;
  aval_s[lane] = a;
  wave_sync();
  return __shfl(incl, kWave - 1, kWave);
}

// index e of the staged entry holding flat product t: pref[e] <= t < pref[e + 1]
__device__ __forceinline__ int staged_entry(const int* pref, int t) {
  int lo = 0, hi = kWave;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pref[mid] <= t)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Visits the staged products t = lane, lane + 64, ... < total, kGather per
// lane at a time: all their B loads are issued before any is used, so a
// wavefront waits for one round of loads per kGather products.
// f(e, q, j, b): staged entry, position in B, column, B value (V = char:
// pattern only, b unused).
constexpr int kGather = 4;
template <typename V, typename F>
__device__ __forceinline__ void for_staged_products(const Problem& pr, int total, const int* start, const int* pref,
                                                    F&& f) {
  const int lane = threadIdx.x & (kWave - 1);
  const V* __restrict__ bval = (const V*)pr.bval;
  for (int t0 = lane; t0 < total; t0 += kGather * kWave) {
    int e[kGather], q[kGather];
    int32_t j[kGather];
    V b[kGather];
#pragma unroll
    for (int u = 0; u < kGather; ++u) {
      const int t = t0 + u * kWave;
      e[u] = -1;
      q[u] = 0;
      j[u] = 0;
      b[u] = V(0);
      if (t < total) {
        e[u] = staged_entry(pref, t);
        q[u] = start[e[u]] + (t - pref[e[u]]);
        j[u] = pr.bci[q[u]];
        if constexpr (!std::is_same<V, char>::value) b[u] = bval[q[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < kGather; ++u)
      if (e[u] >= 0) f(e[u], q[u], j[u], b[u]);
  }
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// ---------------------------------------------------------------- symbolic

// SW: LDS words per wavefront. kSymSlots covers any row (a table, or a d-bit
// bitmap); 2 kHashSplitMin suffices when every row left here has fewer than
// kHashSplitMin products (its table of 2 min(d, flops_i) slots fits).
template <int SW>
__global__ __launch_bounds__(kHashWaves * kWave) void k_hash_symbolic(Problem pr, HashMask hm, HashSplit hs,
                                                                      int32_t* cnt, int32_t* err) {
  __shared__ uint32_t sm[kHashWaves][SW];
  __shared__ int start_s[kHashWaves][kWave], pref_s[kHashWaves][kWave + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  uint32_t* tab = sm[wave];
  int* start = start_s[wave];
  int* pref = pref_s[wave];
  const bool masked = hm.rp || hm.bits;
  for (int64_t row = (int64_t)blockIdx.x * kHashWaves + wave; row < pr.n; row += (int64_t)gridDim.x * kHashWaves) {
    if (hs.slot_of_row[row] >= 0) continue;  // a split row (k_hash_split_claim): the count pass writes cnt
    const int p0 = pr.arp[row], p1 = pr.arp[row + 1];
    const long long fl = pr.flops[row];  // from k_hash_flops
    if (fl == 0) {
      if (lane == 0) cnt[row] = 0;
      continue;
    }
    const int64_t ub = fl < pr.d ? fl : pr.d;
    // up to kRankWords words (d <= 8192) the row's d-bit bitmap is the set
    // (no probing); wider rows use the open-addressing set when it fits
    const bool table = ((pr.d + 31) >> 5) > kRankWords && 2 * ub <= SW;
    const uint32_t tsz = table ? pow2_at_least((uint32_t)(2 * ub)) : 0u;
    const int words = table ? (int)tsz : (pr.d + 31) >> 5;
    for (int t = lane; t < words; t += kWave) tab[t] = table ? kEmpty : 0u;
    wave_sync();
    int fresh = 0;
    for (int base = p0; base < p1; base += kWave) {
      const int nb = min(kWave, p1 - base);
      const int total = stage_products<char>(pr, base, nb, start, pref, nullptr);
      for_staged_products<char>(pr, total, start, pref, [&](int, int, int32_t j, char) {
        if (masked && is_masked(hm, row, j)) return;
        if (table) {
          uint32_t h = hslot(j, tsz - 1);
          uint32_t probes = 0;
          for (;;) {
            const uint32_t old = atomicCAS(&tab[h], kEmpty, (uint32_t)j);
            if (old == kEmpty) {
              ++fresh;
              break;
            }
            if (old == (uint32_t)j) break;
            h = (h + 1) & (tsz - 1);
            if (++probes == tsz) {  // cannot happen: the table has twice the distinct columns
              atomicOr(err, 1);
              break;
            }
          }
        } else {
          const uint32_t bit = 1u << (j & 31);
          if (!(atomicOr(&tab[j >> 5], bit) & bit)) ++fresh;
        }
      });
      wave_sync();
    }
    const long long c = wave_sum_ll(fresh);
    if (lane == 0) cnt[row] = (int32_t)c;
    wave_sync();
  }
}

// Split kernels come in three widths by bitmap words: up to 64 (d <= 2048,
// every row's outputs fit an LDS array of 2048), up to kRankWords and up to
// kSymSlots (LDS arrays of 4096 outputs). Smaller LDS use leaves room for
// more workgroups per CU.
__host__ __device__ constexpr int split_width(int words) {
  return words <= 64 ? 64 : words <= kRankWords ? kRankWords : kSymSlots;
}
__host__ __device__ constexpr int split_lds_outputs(int width) { return width <= 64 ? 2048 : 4096; }

__device__ __forceinline__ int split_lds(const Problem& pr) { return split_lds_outputs(split_width((pr.d + 31) >> 5)); }

// A entries per numeric chunk of a split row (symbolic chunks are
// kSplitEntries; a numeric chunk is that many consecutive ones): a multiple
// of kSplitEntries, enough that a chunk has at least 8 (d <= 2048) or 4
// products per output the row may have (up to the chunk LDS array), so the
// global adds a multi-chunk row's chunks make are at most an eighth or a
// quarter of its products; at most kSplitMaxEntries, so hubs still spread
// over many workgroups.
constexpr int kSplitMaxEntries = 8 * kSplitEntries;
__device__ __forceinline__ int split_chunk_entries(const Problem& pr, int64_t row) {
  const long long fl = pr.flops[row];
  const long long deg = pr.arp[row + 1] - pr.arp[row];
  long long est = fl < pr.d ? fl : pr.d;
  if (est > split_lds(pr)) est = split_lds(pr);
  const long long per = split_lds(pr) <= 2048 ? 8 : 4;  // products per output (measured per width)
  long long e = fl > 0 ? (per * est * deg + fl - 1) / fl : kSplitEntries;
  e = (e + kSplitEntries - 1) / kSplitEntries * kSplitEntries;
  if (e < kSplitEntries) e = kSplitEntries;
  if (e > kSplitMaxEntries) e = kSplitMaxEntries;
  return (int)e;
}

// A split row of one chunk whose outputs fit the chunk's LDS array: the
// chunk writes the row itself (value semirings).
__device__ __forceinline__ bool split_direct(const Problem& pr, int row, int cnt) {
  return pr.arp[row + 1] - pr.arp[row] <= split_chunk_entries(pr, row) && cnt <= split_lds(pr);
}

// A split row with more outputs than that array: written window by window.
__device__ __forceinline__ bool split_windowed(const Problem& pr, int cnt) { return cnt > split_lds(pr); }

// Sum over A entries [p0, p1) of their B row lengths, one wavefront, U
// entries per lane in flight.
template <int U>
__device__ __forceinline__ long long wave_row_flops(const Problem& pr, int p0, int p1) {
  const int lane = threadIdx.x & (kWave - 1);
  long long fl = 0;
  for (int p = p0 + lane; p < p1; p += U * kWave) {
    int k[U];
#pragma unroll
    for (int u = 0; u < U; ++u) k[u] = p + u * kWave < p1 ? pr.aci[p + u * kWave] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k[u] >= 0) fl += pr.brp[k[u] + 1] - pr.brp[k[u]];
  }
  return wave_sum_ll(fl);
}

// Products per row (one wavefront per row). A hub row is a serial chain of
// its wavefront's loads, so long rows keep more of them in flight.
__global__ __launch_bounds__(kHashWaves * kWave) void k_hash_flops(Problem pr) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int64_t row = (int64_t)blockIdx.x * kHashWaves + wave;
  if (row >= pr.n) return;
  const int p0 = pr.arp[row], p1 = pr.arp[row + 1];
  const long long fl = p1 - p0 > 2048 ? wave_row_flops<32>(pr, p0, p1) : wave_row_flops<8>(pr, p0, p1);
  if (lane == 0) pr.flops[row] = fl;
}

// Histogram of floor(log2(flops_i)) over rows with at least kHashSplitMin
// products: LDS counts per workgroup, then one global add per non-zero bin
// (global atomics on a few addresses from every row would serialize).
constexpr int kHistBlocks = 256;
__global__ __launch_bounds__(256) void k_hash_hist(Problem pr, int32_t* hist) {
  __shared__ int32_t h[64];
  if (threadIdx.x < 64) h[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < pr.n;
       row += (int64_t)gridDim.x * blockDim.x) {
    const long long fl = pr.flops[row];
    if (fl >= kHashSplitMin) atomicAdd(&h[63 - __clzll(fl)], 1);
  }
  __syncthreads();
  if (threadIdx.x < 64 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Split slots and chunks for the rows with at least split_flops products.
// A workgroup takes 256 rows at a time and reserves their slots, then the
// chunks of those that got one (below cap), with one global add each (global
// atomics from every row on one counter would serialize). Every row's
// slot_of_row is written: its slot, or -1.
__global__ __launch_bounds__(256) void k_hash_split_claim(Problem pr, HashSplit hs) {
  __shared__ int n_rows_s, n_items_s, base_rows_s, base_items_s;
  for (int64_t r0 = (int64_t)blockIdx.x * blockDim.x; r0 < pr.n; r0 += (int64_t)gridDim.x * blockDim.x) {
    if (threadIdx.x == 0) {
      n_rows_s = 0;
      n_items_s = 0;
    }
    __syncthreads();
    const int64_t row = r0 + threadIdx.x;
    const bool cand = row < pr.n && hs.cap > 0 && pr.flops[row] >= hs.split_flops;
    int local = -1;
    if (cand) local = atomicAdd(&n_rows_s, 1);
    __syncthreads();
    if (threadIdx.x == 0 && n_rows_s > 0) base_rows_s = atomicAdd(&hs.ctr->hash_split_rows, n_rows_s);
    __syncthreads();
    const int slot = cand ? base_rows_s + local : -1;
    const bool split = cand && slot < hs.cap;
    int p0 = 0, nch = 0, item_local = 0;
    if (split) {
      p0 = pr.arp[row];
      nch = (pr.arp[row + 1] - p0 + kSplitEntries - 1) / kSplitEntries;
      item_local = atomicAdd(&n_items_s, nch);
    }
    __syncthreads();
    if (threadIdx.x == 0 && n_items_s > 0) base_items_s = atomicAdd(&hs.ctr->hash_split_items, n_items_s);
    __syncthreads();
    if (row < pr.n) hs.slot_of_row[row] = split ? slot : -1;
    if (split) {
      hs.rows[slot] = (int32_t)row;
      const int first = base_items_s + item_local;
      for (int c = 0; c < nch; ++c) hs.items[first + c] = make_int2(slot, p0 + c * kSplitEntries);
    }
    __syncthreads();  // the LDS counters are reset for the next rows
  }
}

// Symbolic chunks of split rows, one per workgroup. The grid is the host's
// bound on the chunk count (hash_split_item_cap); workgroups past the
// actual count exit at once. Chunks differ in products, and the hardware's
// workgroup dispatch balances them without a shared counter.
template <int WC>
__global__ __launch_bounds__(kSplitWaves * kWave) void k_hash_split_symbolic(Problem pr, HashMask hm, HashSplit hs) {
  __shared__ uint32_t bm[WC];
  __shared__ int start_s[kSplitWaves][kWave], pref_s[kSplitWaves][kWave + 1];
  const int wave = threadIdx.x >> 6;
  const int words = (pr.d + 31) >> 5;
  const bool masked = hm.rp || hm.bits;
  const int it = blockIdx.x;
  if (it >= hs.ctr->hash_split_items) return;
  {
    for (int t = threadIdx.x; t < words; t += blockDim.x) bm[t] = 0u;
    __syncthreads();
    const int2 itm = hs.items[it];
    const int row = hs.rows[itm.x];
    const int a1 = min(itm.y + kSplitEntries, pr.arp[row + 1]);
    for (int base = itm.y + wave * kWave; base < a1; base += kSplitEntries) {
      const int nb = min(kWave, a1 - base);
      const int total = stage_products<char>(pr, base, nb, start_s[wave], pref_s[wave], nullptr);
      for_staged_products<char>(pr, total, start_s[wave], pref_s[wave], [&](int, int, int32_t j, char) {
        if (masked && is_masked(hm, row, j)) return;
        atomicOr(&bm[j >> 5], 1u << (j & 31));
      });
    }
    __syncthreads();
    uint32_t* gb = hs.bits + (int64_t)itm.x * words;
    for (int t = threadIdx.x; t < words; t += blockDim.x) {
      const uint32_t w = bm[t];
      if (w) atomicOr(&gb[t], w);
    }
    __syncthreads();
  }
}

// Per split row: output count (cnt), outputs before each bitmap word (pref),
// the row's first accumulator (acc_off) and its output windows. A workgroup
// takes kCountSlots consecutive slots, one wavefront per slot (64 words a
// step, a running carry), and reserves their accumulators and windows with
// one global add each.
constexpr int kCountSlots = 16;
__global__ __launch_bounds__(kSplitWaves * kWave) void k_hash_split_count(Problem pr, HashSplit hs, int32_t* cnt) {
  __shared__ int acc_need[kCountSlots], win_need[kCountSlots];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int words = (pr.d + 31) >> 5;
  const int nsplit = min(hs.ctr->hash_split_rows, hs.cap);
  for (int s0 = blockIdx.x * kCountSlots; s0 < nsplit; s0 += gridDim.x * kCountSlots) {
    const int s1 = min(s0 + kCountSlots, nsplit);
    for (int slot = s0 + wave; slot < s1; slot += kSplitWaves) {
      const uint32_t* gb = hs.bits + (int64_t)slot * words;
      int32_t* gp = hs.pref + (int64_t)slot * words;
      int run = 0;
      for (int w0 = 0; w0 < words; w0 += kWave) {
        const int w = w0 + lane;
        const int c = w < words ? __popc(gb[w]) : 0;
        int incl = c;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const int y = __shfl_up(incl, o, kWave);
          if (lane >= o) incl += y;
        }
        if (w < words) gp[w] = run + incl - c;
        run += __shfl(incl, kWave - 1, kWave);
      }
      if (lane == 0) {
        const int row = hs.rows[slot];
        cnt[row] = run;
        const int lc = split_lds(pr);
        const bool windowed = split_windowed(pr, run);
        win_need[slot - s0] = windowed ? (run + lc - 1) / lc : 0;
        acc_need[slot - s0] = windowed || split_direct(pr, row, run) ? 0 : run;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int a = 0, w = 0;
      for (int i = 0; i < s1 - s0; ++i) {
        a += acc_need[i];
        w += win_need[i];
      }
      int ao = a ? atomicAdd(&hs.ctr->hash_split_acc, a) : 0;
      int wo = w ? atomicAdd(&hs.ctr->hash_win_items, w) : 0;
      for (int i = 0; i < s1 - s0; ++i) {
        const int slot = s0 + i;
        hs.acc_off[slot] = acc_need[i] ? ao : 0;
        ao += acc_need[i];
        for (int k = 0; k < win_need[i]; ++k) hs.wins[wo + k] = make_int2(slot, k);
        wo += win_need[i];
      }
    }
    __syncthreads();
  }
}

// Rows left to the LDS tables (not split, 1 to kHashNumMax outputs) into the
// row list of their size class; reservations per 256 rows and class.
__global__ __launch_bounds__(256) void k_hash_table_bins(Problem pr, HashSplit hs, const int32_t* cnt) {
  __shared__ int n_s[4], base_s[4];
  for (int64_t r0 = (int64_t)blockIdx.x * blockDim.x; r0 < pr.n; r0 += (int64_t)gridDim.x * blockDim.x) {
    if (threadIdx.x < 4) n_s[threadIdx.x] = 0;
    __syncthreads();
    const int64_t row = r0 + threadIdx.x;
    int c = -1, local = 0;
    if (row < pr.n && hs.slot_of_row[row] < 0) {
      const int nz = cnt[row];
      if (nz > 0 && nz <= kHashNumMax) {
        c = nz <= 64 ? 0 : nz <= 128 ? 1 : nz <= 256 ? 2 : 3;
        local = atomicAdd(&n_s[c], 1);
      }
    }
    __syncthreads();
    if (threadIdx.x < 4 && n_s[threadIdx.x]) base_s[threadIdx.x] = atomicAdd(&hs.cls_cnt[threadIdx.x], n_s[threadIdx.x]);
    __syncthreads();
    if (c >= 0) hs.cls_rows[(int64_t)c * pr.n + base_s[c] + local] = (int32_t)row;
    __syncthreads();
  }
}

// Numeric chunks of split rows into two lists by their row's outputs: at
// most kSplitSmall, or more up to the chunk LDS array (windowed rows are left
// out: their windows write them). Reservations per 256 chunks and class.
__global__ __launch_bounds__(256) void k_hash_chunk_bins(Problem pr, HashSplit hs, const int32_t* cnt) {
  __shared__ int n_s[2], base_s[2];
  const int n_items = hs.ctr->hash_split_items;
  const int lc = split_lds(pr);
  for (int i0 = blockIdx.x * blockDim.x; i0 < n_items; i0 += gridDim.x * blockDim.x) {
    if (threadIdx.x < 2) n_s[threadIdx.x] = 0;
    __syncthreads();
    const int i = i0 + threadIdx.x;
    int c = -1, local = 0;
    if (i < n_items) {
      const int2 itm = hs.items[i];
      const int row = hs.rows[itm.x];
      const int nz = cnt[row];
      // symbolic chunks that start a numeric chunk, of rows not written by windows
      if (nz <= lc && (itm.y - pr.arp[row]) % split_chunk_entries(pr, row) == 0) {
        c = nz <= kSplitSmall ? 0 : 1;
        local = atomicAdd(&n_s[c], 1);
      }
    }
    __syncthreads();
    if (threadIdx.x < 2 && n_s[threadIdx.x])
      base_s[threadIdx.x] = atomicAdd(&hs.cls_cnt[4 + threadIdx.x], n_s[threadIdx.x]);
    __syncthreads();
    if (c >= 0) hs.chunk_lists[(int64_t)c * hs.item_cap + base_s[c] + local] = i;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- numeric

// V = float / int32_t (values) or char (pattern only, OR-AND).
template <typename V>
struct HashAcc {
  using type = typename SemiringT<V>::acc;
};
template <>
struct HashAcc<char> {
  using type = int32_t;
};

template <typename V>
__device__ __forceinline__ typename HashAcc<V>::type hash_prod(V a, V b) {
  if constexpr (std::is_same<V, char>::value)
    return 0;
  else
    return SemiringT<V>::prod(a, b);
}

// Bitonic sort of n2 (power of two) (key, value) pairs in LDS by key, one
// wavefront.
template <typename Acc>
__device__ __forceinline__ void wave_bitonic(uint32_t* key, Acc* val, int n2) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < n2; i += kWave) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const uint32_t a = key[i], b = key[l];
          if ((a > b) == up) {
            key[i] = b;
            key[l] = a;
            const Acc t = val[i];
            val[i] = val[l];
            val[l] = t;
          }
        }
      }
      wave_sync();
    }
  }
}

// Rows with TSZ/4 < nnz_i <= TSZ/2 outputs (the smallest class from one
// output): a table of at most TSZ slots per wavefront.
// RANK: the row is put in column order by each column's rank in an LDS
// bitmap of the row of up to RW words (no sort).
// The rows come from the class's row list (k_hash_table_bins), W wavefronts
// per workgroup, one row each.
template <typename V, int TSZ, bool RANK, int W, int RW_ = kRankWords>
__global__ __launch_bounds__(W * kWave) void k_hash_numeric_table(Problem pr, HashMask hm, const int32_t* list,
                                                                  int32_t count, int32_t* err) {
  using Acc = typename HashAcc<V>::type;
  static_assert(TSZ >= 2 * kWave && TSZ <= kNumSlots, "table class");
  constexpr int RW = RANK ? RW_ : 1;
  __shared__ uint32_t keys_s[W][TSZ];
  __shared__ Acc vals_s[W][TSZ];
  __shared__ int start_s[W][kWave], pref_s[W][kWave + 1];
  __shared__ V aval_s[W][kWave];
  __shared__ uint32_t rbm_s[W][RW];
  __shared__ uint16_t rpw_s[W][RW];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  uint32_t* keys = keys_s[wave];
  Acc* vals = vals_s[wave];
  const bool masked = hm.rp || hm.bits;
  const uint64_t below = lane == 0 ? 0ull : ~0ull >> (kWave - lane);
  for (int64_t i = (int64_t)blockIdx.x * W + wave; i < count; i += (int64_t)gridDim.x * W) {
    const int64_t row = list[i];
    const int c0 = pr.crp[row], nnz = pr.crp[row + 1] - c0;
    if (nnz <= 0 || nnz > TSZ / 2) {  // not this class: the pattern changed since the symbolic call
      if (lane == 0) atomicOr(err, 1);
      continue;
    }
    const uint32_t tsz = pow2_at_least(2u * (uint32_t)nnz);  // <= TSZ
    for (uint32_t t = lane; t < tsz; t += kWave) {
      keys[t] = kEmpty;
      vals[t] = Acc(0);
    }
    wave_sync();
    const int p0 = pr.arp[row], p1 = pr.arp[row + 1];
    for (int base = p0; base < p1; base += kWave) {
      const int nb = min(kWave, p1 - base);
      const int total = stage_products<V>(pr, base, nb, start_s[wave], pref_s[wave], aval_s[wave]);
      for_staged_products<V>(pr, total, start_s[wave], pref_s[wave], [&](int e, int, int32_t j, V b) {
        if (masked && is_masked(hm, row, j)) return;
        uint32_t h = hslot(j, tsz - 1);
        uint32_t probes = 0;
        for (;;) {
          const uint32_t old = atomicCAS(&keys[h], kEmpty, (uint32_t)j);
          if (old == kEmpty || old == (uint32_t)j) break;
          h = (h + 1) & (tsz - 1);
          if (++probes == tsz) {  // more distinct columns than the symbolic count: inputs changed
            atomicOr(err, 1);
            h = kEmpty;
            break;
          }
        }
        if constexpr (!std::is_same<V, char>::value)
          if (h != kEmpty) lds_add(&vals[h], hash_prod<V>(aval_s[wave][e], b));
      });
      wave_sync();
    }
    if constexpr (RANK) {
      // bitmap of the row's columns, outputs before each word, then every
      // occupied slot goes to position (outputs before its word) + (set bits
      // below it in the word)
      uint32_t* bm = rbm_s[wave];
      uint16_t* pw = rpw_s[wave];
      const int words = (pr.d + 31) >> 5;
      for (int w = lane; w < words; w += kWave) bm[w] = 0u;
      wave_sync();
      for (uint32_t t = lane; t < tsz; t += kWave) {
        const uint32_t k = keys[t];
        if (k != kEmpty) atomicOr(&bm[k >> 5], 1u << (k & 31));
      }
      wave_sync();
      if constexpr (RW <= kRankWords) {  // a lane's words at once, one scan
        constexpr int WPL = RW / kWave;    // words per lane
        int cw[WPL], sum = 0;
#pragma unroll
        for (int u = 0; u < WPL; ++u) {
          const int w = lane * WPL + u;
          cw[u] = w < words ? __popc(bm[w]) : 0;
          sum += cw[u];
        }
        int incl = sum;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const int y = __shfl_up(incl, o, kWave);
          if (lane >= o) incl += y;
        }
        int run = incl - sum;
#pragma unroll
        for (int u = 0; u < WPL; ++u) {
          const int w = lane * WPL + u;
          if (w < words) pw[w] = (uint16_t)run;
          run += cw[u];
        }
        if (lane == kWave - 1 && incl != nnz) atomicOr(err, 1);
      } else {  // wide rows: 64 words a step, a running carry
        int run = 0;
        for (int w0 = 0; w0 < words; w0 += kWave) {
          const int w = w0 + lane;
          const int c = w < words ? __popc(bm[w]) : 0;
          int incl = c;
#pragma unroll
          for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
          }
          if (w < words) pw[w] = (uint16_t)(run + incl - c);
          run += __shfl(incl, kWave - 1, kWave);
        }
        if (lane == 0 && run != nnz) atomicOr(err, 1);
      }
      wave_sync();
      for (uint32_t t = lane; t < tsz; t += kWave) {
        const uint32_t k = keys[t];
        if (k == kEmpty) continue;
        const int pos = pw[k >> 5] + __popc(bm[k >> 5] & ((1u << (k & 31)) - 1u));
        if (pos < nnz) {
          pr.cci[c0 + pos] = (int32_t)k;
          if constexpr (!std::is_same<V, char>::value) ((V*)pr.cval)[c0 + pos] = SemiringT<V>::out(vals[t]);
        }
      }
      wave_sync();
      continue;
    }
    // compact the occupied slots to the front (in slot order; every slot is
    // read before any of its block is written), then sort nnz_i of them
    int used = 0;
    for (uint32_t c = 0; c < tsz; c += kWave) {
      const uint32_t key = keys[c + lane];
      const Acc v = vals[c + lane];
      const bool occ = key != kEmpty;
      const uint64_t bal = __ballot(occ);
      const int pos = used + __popcll(bal & below);
      wave_sync();
      if (occ) {
        keys[pos] = key;
        vals[pos] = v;
      }
      used += __popcll(bal);
      wave_sync();
    }
    if (used != nnz && lane == 0) atomicOr(err, 1);
    const uint32_t p2 = pow2_at_least((uint32_t)nnz);
    for (uint32_t t = (uint32_t)used + lane; t < p2; t += kWave) keys[t] = kEmpty;
    wave_sync();
    wave_bitonic<Acc>(keys, vals, (int)p2);
    for (int t = lane; t < nnz; t += kWave) {
      pr.cci[c0 + t] = (int32_t)keys[t];
      if constexpr (!std::is_same<V, char>::value) ((V*)pr.cval)[c0 + t] = SemiringT<V>::out(vals[t]);
    }
    wave_sync();
  }
}

// Rows with more than kHashNumMax outputs: LDS bitmap of d bits, private
// d-wide strip in global memory (kept all-zero between rows).
template <typename V>
__global__ __launch_bounds__(kHashWaves * kWave) void k_hash_numeric_dense(Problem pr, HashMask hm,
                                                                           const int32_t* slot_of_row,
                                                                           typename HashAcc<V>::type* strips,
                                                                           int32_t* err, int32_t* next) {
  using Acc = typename HashAcc<V>::type;
  __shared__ uint32_t bm_s[kHashWaves][kSymSlots];
  __shared__ int start_s[kHashWaves][kWave], pref_s[kHashWaves][kWave + 1];
  __shared__ V aval_s[kHashWaves][kWave];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  uint32_t* bm = bm_s[wave];
  const int words = (pr.d + 31) >> 5;
  Acc* strip = strips + ((int64_t)blockIdx.x * kHashWaves + wave) * pr.d;
  const bool masked = hm.rp || hm.bits;
  for (int t = lane; t < words; t += kWave) bm[t] = 0u;
  wave_sync();
  // rows are taken kDenseFetch at a time from a shared counter (the workers
  // are bounded by their private strips, so a static stride would leave the
  // heavy rows of power-law inputs to a few of them)
  int64_t row = 0, row_end = 0;
  for (;;) {
    if (row == row_end) {
      int c = 0;
      if (lane == 0) c = atomicAdd(next, 1);
      c = __shfl(c, 0, kWave);
      row = (int64_t)c * kDenseFetch;
      if (row >= pr.n) break;
      row_end = row + kDenseFetch < pr.n ? row + kDenseFetch : pr.n;
    }
    const int64_t r = row++;
    const int c0 = pr.crp[r], nnz = pr.crp[r + 1] - c0;
    if (nnz <= kHashNumMax || slot_of_row[r] >= 0) continue;
    const int64_t row_id = r;
    const int p0 = pr.arp[row_id], p1 = pr.arp[row_id + 1];
    for (int base = p0; base < p1; base += kWave) {
      const int nb = min(kWave, p1 - base);
      const int total = stage_products<V>(pr, base, nb, start_s[wave], pref_s[wave], aval_s[wave]);
      for_staged_products<V>(pr, total, start_s[wave], pref_s[wave], [&](int e, int, int32_t j, V b) {
        if (masked && is_masked(hm, row_id, j)) return;
        atomicOr(&bm[j >> 5], 1u << (j & 31));
        if constexpr (!std::is_same<V, char>::value) {
          if constexpr (sizeof(Acc) == 8)
            atomicAdd(&strip[j], hash_prod<V>(aval_s[wave][e], b));
          else
            atomicAdd((unsigned int*)&strip[j], (unsigned int)hash_prod<V>(aval_s[wave][e], b));
        }
      });
      wave_sync();
    }
    __threadfence_block();  // this wavefront's adds are done before they are read back
    // walk the bitmap in 64-word chunks: lane = word, positions by a scan of popcounts
    int base_pos = 0;
    for (int w0 = 0; w0 < words; w0 += kWave) {
      const int w = w0 + lane;
      uint32_t word = w < words ? bm[w] : 0u;
      const int c = __popc(word);
      int incl = c;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
      }
      int pos = c0 + base_pos + incl - c;
      while (word) {
        const int b = __ffs(word) - 1;
        word &= word - 1;
        const int j = (w << 5) + b;
        Acc v = Acc(0);
        if constexpr (!std::is_same<V, char>::value) {
          // read and clear at L2, where the atomic adds landed
          if constexpr (sizeof(Acc) == 8)
            v = __longlong_as_double((long long)atomicExch((unsigned long long*)&strip[j], 0ull));
          else
            v = (Acc)atomicExch((unsigned int*)&strip[j], 0u);
        }
        if (pos < c0 + nnz) {
          pr.cci[pos] = j;
          if constexpr (!std::is_same<V, char>::value) ((V*)pr.cval)[pos] = SemiringT<V>::out(v);
        }
        ++pos;
      }
      if (w < words) bm[w] = 0u;
      base_pos += __shfl(incl, kWave - 1, kWave);
    }
    if (base_pos != nnz && lane == 0) atomicOr(err, 1);
    wave_sync();
  }
}

template <typename A>
__device__ __forceinline__ void global_add(A* p, A v) {
  if constexpr (sizeof(A) == 8)
    atomicAdd(p, v);
  else
    atomicAdd((unsigned int*)p, (unsigned int)v);
}

// Numeric chunk of a split row (one workgroup per chunk). The accumulators
// are zero when it starts; the chunks of a row add in any order.
// LC: outputs of the LDS array; chunks come from the list of their class
// (k_hash_chunk_bins), so every row here has at most LC outputs.
template <typename V, int WC, int LC>
__global__ __launch_bounds__(kSplitWaves * kWave) void k_hash_split_numeric(Problem pr, HashMask hm, HashSplit hs,
                                                                            const int32_t* list, int32_t* err) {
  using Acc = typename HashAcc<V>::type;
  __shared__ uint32_t bm[WC];
  __shared__ int32_t bp[WC];
  __shared__ Acc acc[LC];
  __shared__ int start_s[kSplitWaves][kWave], pref_s[kSplitWaves][kWave + 1];
  __shared__ V aval_s[kSplitWaves][kWave];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int words = (pr.d + 31) >> 5;
  const int2 itm = hs.items[list[blockIdx.x]];
  const int row = hs.rows[itm.x];
  const int cnt = pr.crp[row + 1] - pr.crp[row];
  if (cnt > LC) {  // not this class: the pattern changed since the symbolic call
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  const uint32_t* gb = hs.bits + (int64_t)itm.x * words;
  const int32_t* gp = hs.pref + (int64_t)itm.x * words;
  Acc* gacc = (Acc*)hs.acc + hs.acc_off[itm.x];
  for (int t = threadIdx.x; t < words; t += blockDim.x) {
    bm[t] = gb[t];
    bp[t] = gp[t];
  }
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) acc[t] = Acc(0);
  __syncthreads();
  const bool masked = hm.rp || hm.bits;
  const V* __restrict__ bval = (const V*)pr.bval;
  const int a1 = min(itm.y + split_chunk_entries(pr, row), pr.arp[row + 1]);
  for (int base = itm.y + wave * kWave; base < a1; base += kSplitEntries) {
    const int nb = min(kWave, a1 - base);
    const int total = stage_products<V>(pr, base, nb, start_s[wave], pref_s[wave], aval_s[wave]);
    // U products per lane per step; the next step's B loads are issued before
    // this step's adds, so waiting for them does not wait for the adds
    constexpr int U = 4;
    int en[U];
    int32_t jn[U];
    V bn[U];
    auto load = [&](int t0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + u * kWave;
        en[u] = -1;
        if (t < total) {
          const int e = staged_entry(pref_s[wave], t);
          const int q = start_s[wave][e] + (t - pref_s[wave][e]);
          en[u] = e;
          jn[u] = pr.bci[q];
          bn[u] = bval[q];
        }
      }
    };
    load(lane);
    for (int t0 = lane; t0 < total; t0 += U * kWave) {
      int ec[U];
      int32_t jc[U];
      V bc[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ec[u] = en[u];
        jc[u] = jn[u];
        bc[u] = bn[u];
      }
      load(t0 + U * kWave);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (ec[u] < 0) continue;
        const int32_t j = jc[u];
        if (masked && is_masked(hm, row, j)) continue;
        const uint32_t word = bm[j >> 5], bit = 1u << (j & 31);
        if (!(word & bit)) {  // a column the symbolic phase did not see: inputs changed
          atomicOr(err, 1);
          continue;
        }
        const int pos = bp[j >> 5] + __popc(word & (bit - 1u));
        lds_add(&acc[pos], hash_prod<V>(aval_s[wave][ec[u]], bc[u]));
      }
    }
  }
  __syncthreads();
  if (split_direct(pr, row, cnt)) {  // the whole row: write it in column order
    const int c0 = pr.crp[row];
    for (int w = threadIdx.x; w < words; w += blockDim.x) {
      uint32_t word = bm[w];
      int pos = bp[w];
      while (word) {
        const int b = __ffs(word) - 1;
        word &= word - 1;
        pr.cci[c0 + pos] = (w << 5) + b;
        ((V*)pr.cval)[c0 + pos] = SemiringT<V>::out(acc[pos]);
        ++pos;
      }
    }
    return;
  }
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
    const Acc v = acc[t];
    if (v != Acc(0)) global_add(&gacc[t], v);
  }
}

// One window of output positions [w LC, (w + 1) LC) of a wide split row
// (one workgroup per window). The window's columns are [c_lo, c_hi) (the
// columns at positions lo and hi in the row's bitmap); B rows are sorted, so
// each A entry's products in the window are one range of its B row, found by
// binary search. Those products are added in LDS, then the window is written.
template <typename V, int WC>
__global__ __launch_bounds__(kWinWaves * kWave) void k_hash_split_window(Problem pr, HashMask hm, HashSplit hs,
                                                                         int32_t* err) {
  using Acc = typename HashAcc<V>::type;
  constexpr int LC = split_lds_outputs(WC);
  __shared__ uint32_t bm[WC];
  __shared__ int32_t bp[WC];
  __shared__ Acc acc[LC];
  __shared__ int start_s[kWinWaves][kWave], pref_s[kWinWaves][kWave + 1];
  __shared__ V aval_s[kWinWaves][kWave];
  __shared__ int cols_s[2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int words = (pr.d + 31) >> 5;
  const int2 wi = hs.wins[blockIdx.x];
  const int row = hs.rows[wi.x];
  const int c0 = pr.crp[row], cnt = pr.crp[row + 1] - c0;
  const int lo = wi.y * LC, hi = min(lo + LC, cnt);
  const uint32_t* gb = hs.bits + (int64_t)wi.x * words;
  const int32_t* gp = hs.pref + (int64_t)wi.x * words;
  if (threadIdx.x == 0 && hi == cnt) cols_s[1] = pr.d;  // the last window: up to the last column
  for (int t = threadIdx.x; t < words; t += blockDim.x) {
    uint32_t word = gb[t];
    const int pos = gp[t];
    bm[t] = word;
    bp[t] = pos;
    // the word holding position lo (or hi) gives c_lo (or c_hi)
    const int c = __popc(word);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int target = side ? hi : lo;
      if ((side == 0 || hi < cnt) && pos <= target && target < pos + c) {
        uint32_t x = word;
        for (int k = target - pos; k > 0; --k) x &= x - 1;
        cols_s[side] = (t << 5) + __ffs(x) - 1;
      }
    }
  }
  for (int t = threadIdx.x; t < hi - lo; t += blockDim.x) acc[t] = Acc(0);
  __syncthreads();
  const int c_lo = cols_s[0], c_hi = cols_s[1];
  const bool masked = hm.rp || hm.bits;
  const V* __restrict__ bval = (const V*)pr.bval;
  const int p1 = pr.arp[row + 1];
  for (int base = pr.arp[row] + wave * kWave; base < p1; base += kWinWaves * kWave) {
    const int nb = min(kWave, p1 - base);
    const int total = stage_window(pr, base, nb, c_lo, c_hi, lo == 0, hi == cnt, start_s[wave], pref_s[wave],
                                   aval_s[wave]);
    constexpr int U = 4;  // products per lane per step, loads first
    int e[U];
    int32_t j[U];
    V b[U];
    for (int t0 = lane; t0 < total; t0 += U * kWave) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + u * kWave;
        e[u] = -1;
        if (t < total) {
          e[u] = staged_entry(pref_s[wave], t);
          const int q = start_s[wave][e[u]] + (t - pref_s[wave][e[u]]);
          j[u] = pr.bci[q];
          b[u] = bval[q];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (e[u] < 0) continue;
        if (masked && is_masked(hm, row, j[u])) continue;
        const uint32_t word = bm[j[u] >> 5], bit = 1u << (j[u] & 31);
        if (!(word & bit)) {  // a column the symbolic phase did not see: inputs changed
          atomicOr(err, 1);
          continue;
        }
        const int pos = bp[j[u] >> 5] + __popc(word & (bit - 1u));
        if (pos >= lo && pos < hi) lds_add(&acc[pos - lo], hash_prod<V>(aval_s[wave][e[u]], b[u]));
      }
    }
    wave_sync();  // the staging arrays are rewritten by the next batch
  }
  __syncthreads();
  for (int w = threadIdx.x; w < words; w += blockDim.x) {
    uint32_t word = bm[w];
    int pos = bp[w];
    if (pos >= hi || pos + __popc(word) <= lo) continue;
    while (word) {
      const int bb = __ffs(word) - 1;
      word &= word - 1;
      if (pos >= lo && pos < hi) {
        pr.cci[c0 + pos] = (w << 5) + bb;
        ((V*)pr.cval)[c0 + pos] = SemiringT<V>::out(acc[pos - lo]);
      }
      ++pos;
    }
  }
}

// Writes a split row (one workgroup per row): columns in bitmap order and,
// for value semirings, the row's accumulators.
template <typename V>
__global__ __launch_bounds__(kSplitWaves * kWave) void k_hash_split_emit(Problem pr, HashSplit hs) {
  using Acc = typename HashAcc<V>::type;
  const int slot = blockIdx.x;
  const int words = (pr.d + 31) >> 5;
  const int row = hs.rows[slot];
  const int c0 = pr.crp[row];
  if constexpr (!std::is_same<V, char>::value) {
    const int cnt = pr.crp[row + 1] - c0;
    if (split_direct(pr, row, cnt) || split_windowed(pr, cnt)) return;  // written by its chunk or windows
  }
  const uint32_t* gb = hs.bits + (int64_t)slot * words;
  const int32_t* gp = hs.pref + (int64_t)slot * words;
  const Acc* gacc = (const Acc*)hs.acc + hs.acc_off[slot];
  for (int w = threadIdx.x; w < words; w += blockDim.x) {
    uint32_t word = gb[w];
    int pos = gp[w];
    while (word) {
      const int b = __ffs(word) - 1;
      word &= word - 1;
      pr.cci[c0 + pos] = (w << 5) + b;
      if constexpr (!std::is_same<V, char>::value) ((V*)pr.cval)[c0 + pos] = SemiringT<V>::out(gacc[pos]);
      ++pos;
    }
  }
}

// ---------------------------------------------------------------- launch

int64_t hash_split_candidates(const int32_t* hist) {
  int64_t c = 0;
  for (int b = 63 - __builtin_clzll((unsigned long long)kHashSplitMin); b < 64; ++b) c += hist[b];
  return c;
}

void hash_split_choose(const int32_t* hist, int64_t d, int64_t* split_flops, int64_t* rows) {
  // bitmap and per-word counts: 8 bytes per word and split row, at most 1 GB
  const int64_t words = (d + 31) / 32;
  const int64_t max_rows = (int64_t)(1ll << 30) / (words * 8);
  int t = 63 - __builtin_clzll((unsigned long long)kHashSplitMin);
  int64_t above = 0;
  for (int b = t; b < 64; ++b) above += hist[b];
  while (above > max_rows && t < 63) above -= hist[t++];
  int64_t cap = above;
  if (const char* e = std::getenv("TSSPGEMM_HASH_SPLIT_CAP")) {  // tests: leave split candidates unsplit
    const long long v = std::atoll(e);
    if (v >= 0 && v < cap) cap = v;
  }
  *split_flops = 1ll << t;
  *rows = cap;
}

int64_t hash_split_window_cap(int64_t cap, int64_t d) {
  // a row has at most d outputs: ceil(d / LC) windows
  const int64_t lc = split_lds_outputs(split_width((int)((d + 31) / 32)));
  return cap * ((d + lc - 1) / lc);
}

int64_t hash_split_item_cap(int64_t a_nnz, int64_t cap) {
  // a row of deg A entries makes ceil(deg / kSplitEntries) <= deg / kSplitEntries + 1 chunks
  return a_nnz / kSplitEntries + cap + 1;
}

// One wavefront per row (no grid stride), so the hardware's workgroup
// dispatch balances rows of very different lengths.
int launch_hash_flops(const Problem& pr, int32_t* hist, hipStream_t st) {
  if (pr.n == 0) return TSSPGEMM_OK;
  const int64_t g = (pr.n + kHashWaves - 1) / kHashWaves;
  k_hash_flops<<<(unsigned)g, kHashWaves * kWave, 0, st>>>(pr);
  k_hash_hist<<<kHistBlocks, 256, 0, st>>>(pr, hist);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

int launch_hash_symbolic(const Problem& pr, const HashMask& m, const HashSplit& hs, bool small_rows_only,
                         int32_t* cnt, int32_t* err, hipStream_t st) {
  if (pr.n == 0) return TSSPGEMM_OK;
  // every row's split slot (or -1) first: the short-row kernel skips split rows
  if (hs.cap > 0) {
    const int64_t words = (pr.d + 31) >> 5;
    int rc = launch_zero_bytes(hs.bits, (size_t)hs.cap * words * 4, st);
    if (rc) return rc;
  }
  {
    int64_t gcl = (pr.n + 255) / 256;
    if (gcl > 1024) gcl = 1024;
    k_hash_split_claim<<<(unsigned)gcl, 256, 0, st>>>(pr, hs);
    TSS_CHECK_LAUNCH();
  }
  const int64_t g = (pr.n + kHashWaves - 1) / kHashWaves;
  if (!small_rows_only)
    k_hash_symbolic<kSymSlots><<<(unsigned)g, kHashWaves * kWave, 0, st>>>(pr, m, hs, cnt, err);
  else
    k_hash_symbolic<2 * kHashSplitMin><<<(unsigned)g, kHashWaves * kWave, 0, st>>>(pr, m, hs, cnt, err);
  TSS_CHECK_LAUNCH();
  if (hs.cap > 0) {
    const int wc = split_width((pr.d + 31) >> 5);
    const unsigned gi = (unsigned)hs.item_cap;
    if (wc == 64)
      k_hash_split_symbolic<64><<<gi, kSplitWaves * kWave, 0, st>>>(pr, m, hs);
    else if (wc == kRankWords)
      k_hash_split_symbolic<kRankWords><<<gi, kSplitWaves * kWave, 0, st>>>(pr, m, hs);
    else
      k_hash_split_symbolic<kSymSlots><<<gi, kSplitWaves * kWave, 0, st>>>(pr, m, hs);
    int64_t gc = (hs.cap + kCountSlots - 1) / kCountSlots;
    if (gc > 4096) gc = 4096;
    k_hash_split_count<<<(unsigned)gc, kSplitWaves * kWave, 0, st>>>(pr, hs, cnt);
    TSS_CHECK_LAUNCH();
  }
  int rc = launch_zero_bytes(hs.cls_cnt, 24, st);
  if (rc) return rc;
  int64_t gb = (pr.n + 255) / 256;
  if (gb > 1024) gb = 1024;
  k_hash_table_bins<<<(unsigned)gb, 256, 0, st>>>(pr, hs, cnt);
  if (hs.cap > 0) k_hash_chunk_bins<<<1024, 256, 0, st>>>(pr, hs, cnt);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

int64_t hash_dense_workers(int64_t d) {
  // private strips of d FP64 sums, at most 256 MB in all, whole workgroups
  int64_t w = (int64_t)(256ll << 20) / (d * 8);
  if (w > 1024) w = 1024;
  w = (w / kHashWaves) * kHashWaves;
  return w < kHashWaves ? kHashWaves : w;
}

template <typename V, int TSZ, bool RANK, int W, int RW = kRankWords>
static void table_class(const Problem& pr, const HashMask& h, const HashSplit& hs, int c, const int32_t* cls_n,
                        int32_t* err, hipStream_t st) {
  if (cls_n[c] == 0) return;
  const unsigned g = (unsigned)((cls_n[c] + W - 1) / W);
  k_hash_numeric_table<V, TSZ, RANK, W, RW><<<g, W * kWave, 0, st>>>(pr, h, hs.cls_rows + (int64_t)c * pr.n,
                                                                     cls_n[c], err);
}

// One launch per size class, over that class's rows only. Fewer wavefronts
// share a workgroup as the tables grow, so LDS is allocated in smaller
// pieces (more resident wavefronts per CU).
// Narrow d (RANK): every class orders by rank in a row bitmap. Wide d: the
// two smaller classes sort; the two larger ones rank in a bitmap of up to
// kSymSlots words (LDS for fewer resident wavefronts, but a sort of 256 or
// 512 keys takes dozens of LDS passes).
template <typename V, bool RANK>
static void table_classes(const Problem& pr, const HashMask& h, const HashSplit& hs, const int32_t* cls_n,
                          int32_t* err, hipStream_t st) {
  table_class<V, 128, RANK, 4>(pr, h, hs, 0, cls_n, err, st);
  table_class<V, 256, RANK, 4>(pr, h, hs, 1, cls_n, err, st);
  if constexpr (RANK) {
    table_class<V, 512, true, 2>(pr, h, hs, 2, cls_n, err, st);
    table_class<V, kNumSlots, true, 1>(pr, h, hs, 3, cls_n, err, st);
  } else {
    table_class<V, 512, true, 2, kSymSlots>(pr, h, hs, 2, cls_n, err, st);
    table_class<V, kNumSlots, true, 1, kSymSlots>(pr, h, hs, 3, cls_n, err, st);
  }
}

template <typename V, typename Acc>
static void hash_numeric_kernels(const Problem& pr, const HashMask& h, const HashSplit& hs, int32_t split_rows,
                                 int32_t split_items, int32_t win_items, const int32_t* cls_n, int64_t gd,
                                 void* strips, int32_t* err, int32_t* next, hipStream_t st) {
  const bool narrow = ((pr.d + 31) >> 5) <= kRankWords;
  if (narrow) {
    table_classes<V, true>(pr, h, hs, cls_n, err, st);
  } else {
    table_classes<V, false>(pr, h, hs, cls_n, err, st);
  }
  if (gd > 0)
    k_hash_numeric_dense<V><<<(unsigned)gd, kHashWaves * kWave, 0, st>>>(pr, h, hs.slot_of_row, (Acc*)strips, err,
                                                                          next);
  if constexpr (!std::is_same<V, char>::value) {  // pattern-only rows need no accumulation
    const int wc = split_width((pr.d + 31) >> 5);
    const int32_t* small = hs.chunk_lists;
    const int32_t* large = hs.chunk_lists + hs.item_cap;
    const unsigned gs = (unsigned)cls_n[4], gl = (unsigned)cls_n[5];
    if (wc == 64) {
      if (gs) k_hash_split_numeric<V, 64, kSplitSmall><<<gs, kSplitWaves * kWave, 0, st>>>(pr, h, hs, small, err);
      if (gl) k_hash_split_numeric<V, 64, split_lds_outputs(64)><<<gl, kSplitWaves * kWave, 0, st>>>(pr, h, hs, large, err);
    } else if (wc == kRankWords) {
      if (gs)
        k_hash_split_numeric<V, kRankWords, kSplitSmall><<<gs, kSplitWaves * kWave, 0, st>>>(pr, h, hs, small, err);
      if (gl)
        k_hash_split_numeric<V, kRankWords, split_lds_outputs(kRankWords)>
            <<<gl, kSplitWaves * kWave, 0, st>>>(pr, h, hs, large, err);
    } else {
      if (gs)
        k_hash_split_numeric<V, kSymSlots, kSplitSmall><<<gs, kSplitWaves * kWave, 0, st>>>(pr, h, hs, small, err);
      if (gl)
        k_hash_split_numeric<V, kSymSlots, split_lds_outputs(kSymSlots)>
            <<<gl, kSplitWaves * kWave, 0, st>>>(pr, h, hs, large, err);
    }
    const unsigned gw = (unsigned)win_items;
    if (win_items > 0 && wc == 64)
      k_hash_split_window<V, 64><<<gw, kWinWaves * kWave, 0, st>>>(pr, h, hs, err);
    else if (win_items > 0 && wc == kRankWords)
      k_hash_split_window<V, kRankWords><<<gw, kWinWaves * kWave, 0, st>>>(pr, h, hs, err);
    else if (win_items > 0)
      k_hash_split_window<V, kSymSlots><<<gw, kWinWaves * kWave, 0, st>>>(pr, h, hs, err);
  }
  if (split_rows > 0) k_hash_split_emit<V><<<(unsigned)split_rows, kSplitWaves * kWave, 0, st>>>(pr, hs);
}

int launch_hash_numeric(int sr, const Problem& pr, const HashMask& h, const HashSplit& hs, int32_t split_rows,
                        int32_t split_items, int64_t split_acc, int32_t win_items, const int32_t* cls_n,
                        bool long_rows, void* strips, int32_t* err, int32_t* next, hipStream_t st) {
  if (pr.n == 0) return TSSPGEMM_OK;
  const int64_t g = (pr.n + kHashWaves - 1) / kHashWaves;  // the long-row workers never outnumber the rows
  int64_t gd = long_rows ? hash_dense_workers(pr.d) / kHashWaves : 0;  // long-row workers, if any row needs them
  if (gd > g) gd = g;
  int rc;
  if ((rc = launch_zero_bytes(next, 4, st))) return rc;
  const size_t acc_bytes = sr == TSSPGEMM_PLUS_TIMES_F32 ? 8 : 4;
  if (sr != TSSPGEMM_OR_AND && split_acc > 0 && (rc = launch_zero_bytes(hs.acc, (size_t)split_acc * acc_bytes, st)))
    return rc;
  if (sr == TSSPGEMM_PLUS_TIMES_F32)
    hash_numeric_kernels<float, double>(pr, h, hs, split_rows, split_items, win_items, cls_n, gd, strips, err,
                                        next, st);
  else if (sr == TSSPGEMM_PLUS_TIMES_I32)
    hash_numeric_kernels<int32_t, int32_t>(pr, h, hs, split_rows, split_items, win_items, cls_n, gd, strips,
                                          err, next, st);
  else
    hash_numeric_kernels<char, int32_t>(pr, h, hs, split_rows, split_items, win_items, cls_n, gd, strips, err,
                                       next, st);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

}  // namespace tss
