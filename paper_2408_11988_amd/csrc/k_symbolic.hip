// Symbolic phase of row-wise Gustavson TS-SpGEMM (Sec. III-A, Eq. 1): for
// every row i, flops_i = number of products A(i,k) B(k,j) (Sec. II-A) and the
// output pattern pat(C_i) = union of pat(B_k) over k in pat(A_i), minus an
// optional complement mask (Algorithm 3's N \ S). The union is formed in a
// d-bit bitmap per row -- the dense (SPA-like) accumulator of Sec. III-C,
// here held in registers: a slot of `wp` lanes owns one B row's bitmap words,
// a wavefront ORs 64/wp B rows per step and reduces across slots at the end.
//
// Also here: the B-pattern bitmap build, the work binning of rows by A-row
// length, and the popcount + exclusive scan that turns C's bitmaps into
// C's row pointers.
#include "dev_numeric.hpp"
#include "dev_symbolic.hpp"

namespace tss {

// ================================================================ utilities

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

int launch_zero_bytes(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return TSSPGEMM_OK;
  // byte counts used in this library are multiples of 4
  int64_t n = (int64_t)(bytes / 4);
  unsigned g = grid_for(n, 256 * 8);
  if (g > 4096) g = 4096;
  k_zero_u32<<<g, 256, 0, st>>>((uint32_t*)p, n);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

int launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n == 0) return TSSPGEMM_OK;
  unsigned g = grid_for(n, 256 * 8);
  if (g > 8192) g = 8192;
  k_fill_i32<<<g, 256, 0, st>>>(p, n, v);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

__global__ __launch_bounds__(256) void k_csr_to_bitmap(int64_t n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, int wp,
                                                       uint32_t* __restrict__ bits, uint8_t* narrow8,
                                                       uint16_t* narrow16) {
  extern __shared__ __align__(16) uint32_t sm[];
  bitmap_block(n, rp, ci, wp, bits, (int64_t)blockIdx.x * kBmRows, sm, narrow8, narrow16);
}

int launch_csr_to_bitmap(int64_t n, const int32_t* rp, const int32_t* ci, int wp, uint32_t* bits, hipStream_t st,
                         void* narrow, int narrow_bytes) {
  if (n == 0) return TSSPGEMM_OK;
  const size_t lds = (size_t)(kBmRows + 1 + kBmRows * wp) * 4;
  k_csr_to_bitmap<<<grid_for(n, kBmRows), 256, lds, st>>>(n, rp, ci, wp, bits,
                                                          narrow_bytes == 1 ? (uint8_t*)narrow : nullptr,
                                                          narrow_bytes == 2 ? (uint16_t*)narrow : nullptr);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// bit r of `bits` = row r of the CSR is non-empty
__global__ void k_nonempty_bits(int64_t n, const int32_t* __restrict__ rp, uint32_t* __restrict__ bits) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  bool ne = r < n && rp[r + 1] > rp[r];
  uint64_t b = __ballot(ne);
  if ((threadIdx.x & 63) == 0 && r < n) {
    int64_t w = r >> 5;  // r is a multiple of 64 here
    bits[w] = (uint32_t)b;
    if (r + 32 < n) bits[w + 1] = (uint32_t)(b >> 32);
  }
}

int launch_nonempty_bits(int64_t n, const int32_t* rp, uint32_t* bits, hipStream_t st) {
  if (n == 0) return TSSPGEMM_OK;
  k_nonempty_bits<<<grid_for(n, 256), 256, 0, st>>>(n, rp, bits);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// CSR invariants: rp[0] = 0, rp non-decreasing, rp[n] = nnz, columns strictly
// increasing within a row and inside [0, ncols).
__global__ void k_validate_csr(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t* __restrict__ rp,
                               const int32_t* __restrict__ ci, Counters* ctr) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int a = rp[r], b = rp[r + 1];
  bool bad = (r == 0 && a != 0) || (r == nrows - 1 && b != nnz) || b < a || a < 0 || b > nnz;
  if (!bad) {
    int prev = -1;
    for (int q = a; q < b; ++q) {
      const int j = ci[q];
      if (j <= prev || j >= ncols) {
        bad = true;
        break;
      }
      prev = j;
    }
  }
  if (bad) atomicOr(&ctr->malformed, 1);
}

int launch_validate_csr(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t* rp, const int32_t* ci,
                        Counters* ctr, hipStream_t st) {
  if (nrows == 0) return TSSPGEMM_OK;
  k_validate_csr<<<grid_for(nrows, 256), 256, 0, st>>>(nrows, ncols, nnz, rp, ci, ctr);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// ================================================================ binning (symbolic)

// The rows of one binning workgroup (256 threads, kBinRowsPerBlock rows):
// thread t takes rows r0 + t + 256 u. Their first A entries and A entry
// counts are loaded into registers up front (all loads in flight at once;
// rows past n get 0 entries).
constexpr int kBinThreads = 256;
constexpr int kBinPer = kBinRowsPerBlock / kBinThreads;

__device__ __forceinline__ void bin_rows(const int32_t* __restrict__ arp, int64_t n, int64_t r0, int (&a)[kBinPer],
                                         int (&m)[kBinPer]) {
  int e[kBinPer];
#pragma unroll
  for (int u = 0; u < kBinPer; ++u) {
    const int64_t i = r0 + threadIdx.x + (int64_t)kBinThreads * u;
    a[u] = i < n ? arp[i] : 0;
    e[u] = i < n ? arp[i + 1] : 0;
  }
#pragma unroll
  for (int u = 0; u < kBinPer; ++u) m[u] = e[u] - a[u];
}

__global__ __launch_bounds__(kBinThreads) void k_sym_bin_count(Problem pr, int32_t split_nnz, int32_t light_max,
                                                               Counters* ctr) {
  __shared__ int32_t hist[kBins];
  if (threadIdx.x < kBins) hist[threadIdx.x] = 0;
  int a[kBinPer], m[kBinPer];
  bin_rows(pr.arp, pr.n, (int64_t)blockIdx.x * kBinRowsPerBlock, a, m);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kBinPer; ++u) {
    int bin, count;
    sym_bin(m[u], split_nnz, bin, count, light_max);
    if (count) atomicAdd(&hist[bin], count);
  }
  __syncthreads();
  if (threadIdx.x < kBins && hist[threadIdx.x]) atomicAdd(&ctr->sym_count[threadIdx.x], hist[threadIdx.x]);
}

// Items are placed with one global reservation per bin per workgroup (its
// counts from a first pass over its rows): the bin's offset (a scan of the
// counts, done by every workgroup) plus the bin's fill counter (sym_cursor,
// zero at the start); the slot inside the workgroup's range comes from an
// LDS counter in the second pass. Workgroup 0 stores the item total.
__global__ __launch_bounds__(kBinThreads) void k_sym_bin_fill(Problem pr, int32_t split_nnz, int32_t light_max,
                                                              Item* items, Counters* ctr, bool zero_split) {
  __shared__ int32_t cnt[kBins], base[kBins], off[kBins];
  if (threadIdx.x < kBins) cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    int32_t o = 0;
    for (int b = 0; b < kBins; ++b) {
      off[b] = o;
      o += ctr->sym_count[b];
    }
    if (blockIdx.x == 0) ctr->sym_total = o;
  }
  const int64_t r0 = (int64_t)blockIdx.x * kBinRowsPerBlock;
  int a[kBinPer], m[kBinPer];
  bin_rows(pr.arp, pr.n, r0, a, m);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kBinPer; ++u) {
    int bin, count;
    sym_bin(m[u], split_nnz, bin, count, light_max);
    if (count) atomicAdd(&cnt[bin], count);
  }
  __syncthreads();
  if (threadIdx.x < kBins) {
    if (cnt[threadIdx.x])
      base[threadIdx.x] = off[threadIdx.x] + atomicAdd(&ctr->sym_cursor[threadIdx.x], cnt[threadIdx.x]);
    cnt[threadIdx.x] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kBinPer; ++u) {
    int bin, count;
    sym_bin(m[u], split_nnz, bin, count, light_max);
    if (!count) continue;
    const int64_t i = r0 + threadIdx.x + (int64_t)kBinThreads * u;
    const int pos = base[bin] + atomicAdd(&cnt[bin], count);
    if (m[u] <= split_nnz) {
      items[pos] = Item{(int32_t)i, a[u], a[u] + m[u], 0};
    } else {
      for (int c = 0; c < count; ++c) {
        const int p0 = a[u] + c * split_nnz;
        items[pos + c] = Item{(int32_t)i, p0, min(a[u] + m[u], p0 + split_nnz), kSplitFlag | c};
      }
      if (zero_split) {
        for (int w = 0; w < pr.wp; ++w) pr.cbits[i * pr.wp + w] = 0u;
        pr.flops[i] = 0;
      }
    }
  }
}

int launch_sym_bin(const Problem& pr, int32_t split_nnz, Item* items, Counters* ctr, hipStream_t st,
                   bool zero_split, int32_t light_max) {
  if (pr.n == 0) return TSSPGEMM_OK;  // the zeroed counters are the totals
  const unsigned g = grid_for(pr.n, kBinRowsPerBlock);
  k_sym_bin_count<<<g, kBinThreads, 0, st>>>(pr, split_nnz, light_max, ctr);
  k_sym_bin_fill<<<g, kBinThreads, 0, st>>>(pr, split_nnz, light_max, items, ctr, zero_split);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// ================================================================ symbolic

// Light rows. WP = bitmap words per row (power of two, 1..32); a slot of WP
// lanes owns one row (lane = slot * WP + word) and walks its A entries,
// OR-ing the B rows' bitmap words; 64/WP rows per wavefront are in flight.
template <int WP>
__global__ __launch_bounds__(kBlock) void k_symbolic_light(SymParams sp) {
  constexpr int NS = kWave / WP;
  const Problem& pr = sp.pr;
  const int lane = threadIdx.x & (kWave - 1);
  const int slot = lane / WP, w = lane % WP;
  const int64_t row = ((int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)) * NS + slot;
  const uint32_t* __restrict__ bb = pr.bbits;
  const int32_t* __restrict__ aci = pr.aci;
  if (row >= pr.n) return;
  const int p0 = pr.arp[row], p1 = pr.arp[row + 1];
  if (p1 - p0 > sp.light_max) return;  // a heavy row: done from the item list
  uint32_t mword = 0u, need = 0xffffffffu;
  bool work = p1 > p0;
  if (sp.mask) {
    mword = sp.mask[row * WP + w];
    need = ~mword & (sp.active ? sp.active[w] : 0xffffffffu);
    uint32_t any = need;
#pragma unroll
    for (int o = 1; o < WP; o <<= 1) any |= shfl_xor_u32(any, o);
    work = work && any != 0u;
  }
  uint32_t acc = 0u;
  int fl = 0;
  if (work) {
    const uint32_t* __restrict__ fnz = sp.fnz;
    int p = p0;
    if (fnz == nullptr) {
      for (; p + 3 < p1; p += 4) {
        const int k0 = aci[p], k1 = aci[p + 1], k2 = aci[p + 2], k3 = aci[p + 3];
        const uint32_t x0 = bb[(int64_t)k0 * WP + w], x1 = bb[(int64_t)k1 * WP + w];
        const uint32_t x2 = bb[(int64_t)k2 * WP + w], x3 = bb[(int64_t)k3 * WP + w];
        acc |= (x0 | x1) | (x2 | x3);
        fl += __popc(x0) + __popc(x1) + __popc(x2) + __popc(x3);
      }
      for (; p < p1; ++p) {
        const uint32_t x = bb[(int64_t)aci[p] * WP + w];
        acc |= x;
        fl += __popc(x);
      }
    } else {
      // B rows flagged empty are skipped; four A entries per step, their
      // summary bits and B words loaded together
      const uint64_t smask = (WP >= 64 ? ~0ull : ((1ull << WP) - 1ull)) << (WP >= 64 ? 0 : slot * WP);
      for (; p < p1; p += 4) {
        int k[4];
        bool v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          v[u] = p + u < p1;
          k[u] = v[u] ? aci[p + u] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = v[u] && ((fnz[k[u] >> 5] >> (k[u] & 31)) & 1u);
        uint32_t x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = v[u] ? bb[(int64_t)k[u] * WP + w] : 0u;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          acc |= x[u];
          fl += __popc(x[u]);
        }
        if (sp.early_exit && (__ballot((need & ~acc) != 0u) & smask) == 0ull) break;
      }
    }
  }
#pragma unroll
  for (int o = 1; o < WP; o <<= 1) fl += __shfl_xor(fl, o, kWave);
  pr.cbits[row * WP + w] = acc & ~mword;
  if (w == 0) pr.flops[row] = fl;
}

// Heavy rows and chunks of split rows, from the item list. A wavefront per
// item: lane = slot * WP + word, 64/WP B rows in flight, OR-reduced across
// slots at the end. Wavefronts walk the list with a grid stride; items are
// ordered heaviest first, so every wavefront gets a similar mix.
template <int WP>
__global__ __launch_bounds__(kBlock) void k_symbolic(SymParams sp) {
  constexpr int NS = kWave / WP;  // slots (B rows in flight) per wavefront
  const Problem& pr = sp.pr;
  const int lane = threadIdx.x & (kWave - 1);
  const int slot = lane / WP, w = lane % WP;
  const int total = sp.ctr->sym_total;
  const int wave_global = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int wave_stride = gridDim.x * kWavesPerBlock;
  const uint32_t* __restrict__ bb = sp.pr.bbits;
  const int32_t* __restrict__ aci = pr.aci;
  const uint32_t* __restrict__ fnz = sp.fnz;

  for (int t = wave_global; t < total; t += wave_stride) {
    const Item it = sp.items[t];
    const bool split = (it.aux & kSplitFlag) != 0;
    const int64_t row = it.row;
    uint32_t mword = 0, need = 0xffffffffu;
    bool skip = false;
    if (sp.mask) {
      mword = sp.mask[row * WP + w];
      need = ~mword & (sp.active ? sp.active[w] : 0xffffffffu);
      // every column that could be produced is masked out: nothing to do
      if (!split) skip = __ballot(need != 0u) == 0ull;
    }
    uint32_t acc = 0u;
    int fl = 0;
    if (!skip) {
      if (fnz == nullptr) {
        acc = sym_item_or_slots(pr, it.p0, it.p1, WP, lane, need & word_cols(pr.d, w), fl);
      } else {
        // wavefront-uniform steps of 16 * NS entries (entry base + slot + u NS),
        // so the early-exit test below sees every lane (16 per slot in flight:
        // R-MAT 22 x 512 BFS 18.6 ms, against 19.4 with 8 and 21.1 with 4)
        for (int base = it.p0; base < it.p1; base += 16 * NS) {
          int k[16];
          bool v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int q = base + slot + u * NS;
            v[u] = q < it.p1;
            k[u] = v[u] ? aci[q] : 0;
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) v[u] = v[u] && ((fnz[k[u] >> 5] >> (k[u] & 31)) & 1u);
          uint32_t x[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) x[u] = v[u] ? bb[(int64_t)k[u] * WP + w] : 0u;
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            acc |= x[u];
            fl += __popc(x[u]);
          }
          if (sp.early_exit) {
            uint32_t all = acc;  // this word OR-ed over the slots
#pragma unroll
            for (int o = WP; o < kWave; o <<= 1) all |= shfl_xor_u32(all, o);
            if (__ballot((need & ~all) != 0u) == 0ull) break;
          }
        }
      }
    }
#pragma unroll
    for (int o = WP; o < kWave; o <<= 1) acc |= shfl_xor_u32(acc, o);
    const long long fsum = wave_sum_i64((long long)fl);
    if (slot == 0) {
      if (split) {
        if (acc) atomicOr(&pr.cbits[row * WP + w], acc);
      } else {
        pr.cbits[row * WP + w] = acc & ~mword;
      }
    }
    if (lane == 0) {
      if (split)
        atomicAdd((unsigned long long*)&pr.flops[row], (unsigned long long)fsum);
      else
        pr.flops[row] = fsum;
    }
  }
}

// Unmasked symbolic pass, one lane per A entry: a lane loads the whole
// bitmap row of its entry's B row (WP words, 16-byte loads), so a wavefront
// has 64 B rows per load instruction in flight. Light rows: a lane owns a
// row and walks its entries. Heavy items: the lanes of a wavefront take the
// item's entries in turn and OR their words together, stopping the gathers
// once the row holds every column (sym_item_or).
template <int WP>
__global__ __launch_bounds__(kBlock) void k_symbolic_light_lanes(SymParams sp) {
  const Problem& pr = sp.pr;
  const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (row >= pr.n) return;
  const int p0 = pr.arp[row], p1 = pr.arp[row + 1];
  if (p1 - p0 > sp.light_max) return;  // a heavy row: done from the item list
  const uint32_t* __restrict__ bb = pr.bbits;
  BmRow<WP> acc;
#pragma unroll
  for (int w = 0; w < WP; ++w) acc.w[w] = 0u;
  int fl = 0;
  int p = p0;
  for (; p + 3 < p1; p += 4) {  // four B bitmap rows in flight
    const int k0 = pr.aci[p], k1 = pr.aci[p + 1], k2 = pr.aci[p + 2], k3 = pr.aci[p + 3];
    bm_load_or<WP>(bb + (int64_t)k0 * WP, acc, fl);
    bm_load_or<WP>(bb + (int64_t)k1 * WP, acc, fl);
    bm_load_or<WP>(bb + (int64_t)k2 * WP, acc, fl);
    bm_load_or<WP>(bb + (int64_t)k3 * WP, acc, fl);
  }
  for (; p < p1; ++p) bm_load_or<WP>(bb + (int64_t)pr.aci[p] * WP, acc, fl);
  bm_store<WP>(pr.cbits + row * WP, acc);
  pr.flops[row] = fl;
}

template <int WP>
__global__ __launch_bounds__(kBlock) void k_symbolic_lanes(SymParams sp) {
  const Problem& pr = sp.pr;
  const int lane = threadIdx.x & (kWave - 1);
  const int total = sp.ctr->sym_total;
  const int wave_global = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int wave_stride = gridDim.x * kWavesPerBlock;
  for (int t = wave_global; t < total; t += wave_stride) {
    const Item it = sp.items[t];
    const bool split = (it.aux & kSplitFlag) != 0;
    const int64_t row = it.row;
    int fl = 0;
    const uint32_t word = sym_item_or<WP>(pr, it.p0, it.p1, lane, fl);
    // products: at most 32 * WP per entry, so an int32 sum holds below 2^31 / (32 WP) entries
    const long long fsum = (int64_t)(it.p1 - it.p0) * 32 * WP < (1ll << 31) ? (long long)wave_sum_i32(fl)
                                                                              : wave_sum_i64((long long)fl);
    if ((lane & (kWave / WP - 1)) == 0) {  // the first lane holding each word
      uint32_t* dst = &pr.cbits[row * WP + bm_word_of<WP>(lane)];
      if (split) {
        if (word) atomicOr(dst, word);
      } else {
        *dst = word;
      }
    }
    if (lane == 0) {
      if (split)
        atomicAdd((unsigned long long*)&pr.flops[row], (unsigned long long)fsum);
      else
        pr.flops[row] = fsum;
    }
  }
}

// Masked symbolic pass (a complement mask, optionally the active columns,
// the frontier summary fnz and early exit), one lane per light row or per A
// entry with whole B bitmap rows in registers (at most 16 words): the same
// results as k_symbolic_light / k_symbolic, with 64 rows or entries per
// wavefront in flight instead of 64 / WP. A light row's lane keeps its open
// columns (not masked, active) and stops once its accumulator covers them.
__device__ __forceinline__ bool fnz_set(const uint32_t* fnz, int k) {
  return fnz == nullptr || ((fnz[k >> 5] >> (k & 31)) & 1u);
}

template <int WP>
__global__ __launch_bounds__(kBlock) void k_symbolic_light_lanes_m(SymParams sp) {
  const Problem& pr = sp.pr;
  const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (row >= pr.n) return;
  const int p0 = pr.arp[row], p1 = pr.arp[row + 1];
  if (p1 - p0 > sp.light_max) return;  // a heavy row: done from the item list
  const uint32_t* __restrict__ bb = pr.bbits;
  const uint32_t* __restrict__ fnz = sp.fnz;
  BmRow<WP> need, acc;
  uint32_t open = 0u;
#pragma unroll
  for (int w = 0; w < WP; ++w) {
    const uint32_t m = sp.mask ? sp.mask[row * WP + w] : 0u;
    need.w[w] = ~m & (sp.active ? sp.active[w] : 0xffffffffu);
    open |= need.w[w];
    acc.w[w] = 0u;
  }
  int fl = 0;
  if (p1 > p0 && (sp.mask == nullptr || open != 0u)) {
    for (int p = p0; p < p1; p += 2) {
      const int k0 = pr.aci[p];
      const int k1 = p + 1 < p1 ? pr.aci[p + 1] : -1;
      const bool v0 = fnz_set(fnz, k0), v1 = k1 >= 0 && fnz_set(fnz, k1);
      if (v0) bm_load_or<WP>(bb + (int64_t)k0 * WP, acc, fl);
      if (v1) bm_load_or<WP>(bb + (int64_t)k1 * WP, acc, fl);
      if (sp.early_exit) {
        uint32_t left = 0u;
#pragma unroll
        for (int w = 0; w < WP; ++w) left |= need.w[w] & ~acc.w[w];
        if (left == 0u) break;
      }
    }
  }
#pragma unroll
  for (int w = 0; w < WP; ++w) {
    const uint32_t m = sp.mask ? sp.mask[row * WP + w] : 0u;
    acc.w[w] &= ~m;
  }
  bm_store<WP>(pr.cbits + row * WP, acc);
  pr.flops[row] = fl;
}

template <int WP>
__global__ __launch_bounds__(kBlock) void k_symbolic_lanes_m(SymParams sp) {
  const Problem& pr = sp.pr;
  const int lane = threadIdx.x & (kWave - 1);
  const int total = sp.ctr->sym_total;
  const int wave_global = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int wave_stride = gridDim.x * kWavesPerBlock;
  const uint32_t* __restrict__ bb = pr.bbits;
  const uint32_t* __restrict__ fnz = sp.fnz;
  const int myw = bm_word_of<WP>(lane);  // the word this lane holds after the reduction
  for (int t = wave_global; t < total; t += wave_stride) {
    const Item it = sp.items[t];
    const bool split = (it.aux & kSplitFlag) != 0;
    const int64_t row = it.row;
    const uint32_t mword = sp.mask ? sp.mask[row * WP + myw] : 0u;
    const uint32_t need = ~mword & (sp.active ? sp.active[myw] : 0xffffffffu);
    // every column that could be produced is masked out: nothing to do
    const bool skip = sp.mask && !split && __ballot(need != 0u) == 0ull;
    BmRow<WP> acc;
#pragma unroll
    for (int w = 0; w < WP; ++w) acc.w[w] = 0u;
    int fl = 0;
    if (!skip) {
      for (int base = it.p0; base < it.p1; base += kWave) {  // wavefront-uniform steps
        const int p = base + lane;
        const int k = p < it.p1 ? pr.aci[p] : -1;
        if (k >= 0 && fnz_set(fnz, k)) bm_load_or<WP>(bb + (int64_t)k * WP, acc, fl);
        if (sp.early_exit) {
          const uint32_t word = bm_wave_or<WP>(acc, lane);
          if (__ballot((need & ~word) != 0u) == 0ull) break;
        }
      }
    }
    const uint32_t word = bm_wave_or<WP>(acc, lane);
    const long long fsum = wave_sum_i64((long long)fl);
    if ((lane & (kWave / WP - 1)) == 0) {  // the first lane holding each word
      uint32_t* dst = &pr.cbits[row * WP + myw];
      if (split) {
        if (word) atomicOr(dst, word);
      } else {
        *dst = word & ~mword;
      }
    }
    if (lane == 0) {
      if (split)
        atomicAdd((unsigned long long*)&pr.flops[row], (unsigned long long)fsum);
      else
        pr.flops[row] = fsum;
    }
  }
}

int launch_symbolic(const SymParams& sp, int64_t max_items, hipStream_t st) {
  return launch_symbolic_part(sp, max_items, kSymLight | kSymHeavy, st);
}

int launch_symbolic_part(const SymParams& sp, int64_t max_items, int part, hipStream_t st) {
  const int64_t n = sp.pr.n;
  if (n == 0) return TSSPGEMM_OK;
  const bool do_light = (part & kSymLight) != 0;
  if (!(part & kSymHeavy)) max_items = 0;  // no heavy launch
  const int ns = kWave / sp.pr.wp;
  const unsigned g_light = grid_for(n, ns * kWavesPerBlock);
  // heavy items: a wavefront walks items t, t + waves, ...; eight times the
  // resident wavefronts (256 CUs x 32), so that the dispatcher, starting
  // workgroups as others finish, evens out the items' unequal latency chains
  // (R-MAT 20 x 128 pass: 0.340 ms with one wavefront per resident slot,
  // 0.314 with eight; R-MAT 22 x 512 BFS: 17.0 against 14.9 ms)
  const int64_t waves = max_items < 256 * 256 ? max_items : 256 * 256;
  const unsigned g_heavy = grid_for(waves, kWavesPerBlock);
  // without a mask, and for bitmap rows of at most 8 words (registers): one
  // lane per A entry (k_symbolic_*_lanes)
  const bool lanes = sp.mask == nullptr && sp.fnz == nullptr && sp.pr.wp <= 8;
  // with a mask, or bitmap rows of 16 words: the same lane-per-row /
  // lane-per-entry form with the mask. Heavy items with early exit (the BFS)
  // keep the slot kernel, which tests coverage without a wavefront-wide
  // reduction (R-MAT 22 x 512 BFS: heavy items 0.97 ms per product in slots,
  // 1.81 ms in the lane form; light rows 0.83 ms in slots, 0.48 ms as lanes)
  const bool light_m = !lanes && sp.pr.wp <= 16;
  const bool heavy_m = light_m && !sp.early_exit;
  const unsigned g_lanes = grid_for(n, kBlock);
#define TSS_SYM_CASE(W)                                                           \
  case W:                                                                         \
    if (lanes) {                                                                  \
      if (do_light) k_symbolic_light_lanes<W><<<g_lanes, kBlock, 0, st>>>(sp);    \
      if (max_items > 0) k_symbolic_lanes<W><<<g_heavy, kBlock, 0, st>>>(sp);     \
    } else if (light_m) {                                                         \
      if (do_light)                                                               \
        k_symbolic_light_lanes_m<(W <= 16 ? W : 16)><<<g_lanes, kBlock, 0, st>>>(sp); \
      if (max_items > 0 && heavy_m)                                               \
        k_symbolic_lanes_m<(W <= 16 ? W : 16)><<<g_heavy, kBlock, 0, st>>>(sp);   \
      else if (max_items > 0)                                                     \
        k_symbolic<W><<<g_heavy, kBlock, 0, st>>>(sp);                            \
    } else {                                                                      \
      if (do_light) k_symbolic_light<W><<<g_light, kBlock, 0, st>>>(sp);          \
      if (max_items > 0) k_symbolic<W><<<g_heavy, kBlock, 0, st>>>(sp);           \
    }                                                                             \
    break;
  switch (sp.pr.wp) {
    TSS_SYM_CASE(1)
    TSS_SYM_CASE(2)
    TSS_SYM_CASE(4)
    TSS_SYM_CASE(8)
    TSS_SYM_CASE(16)
    TSS_SYM_CASE(32)
    default: set_error("symbolic: unsupported bitmap width"); return TSSPGEMM_ERR_UNSUPPORTED;
  }
#undef TSS_SYM_CASE
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// Split rows are OR-ed / added chunk by chunk: zero their bitmap row and
// product count first (one thread per item, acting on chunk 0 items).
__global__ void k_sym_split_zero(Problem pr, const Item* items, const Counters* ctr) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ctr->sym_total) return;
  const Item it = items[t];
  if ((it.aux & kSplitFlag) == 0 || (it.aux & ~kSplitFlag) != 0) return;
  for (int w = 0; w < pr.wp; ++w) pr.cbits[(int64_t)it.row * pr.wp + w] = 0u;
  pr.flops[it.row] = 0;
}

int launch_sym_split_zero(const Problem& pr, const Item* items, Counters* ctr, int64_t max_items, hipStream_t st) {
  if (max_items == 0) return TSSPGEMM_OK;
  k_sym_split_zero<<<grid_for(max_items, 256), 256, 0, st>>>(pr, items, ctr);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// Split rows were OR-ed chunk by chunk; apply the complement mask once all
// chunks are in (one thread per split row, found from its chunk 0 item).
__global__ void k_sym_split_mask(Problem pr, const Item* items, const uint32_t* mask, const Counters* ctr) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ctr->sym_total) return;
  const Item it = items[t];
  if ((it.aux & kSplitFlag) == 0 || (it.aux & ~kSplitFlag) != 0) return;
  for (int w = 0; w < pr.wp; ++w) pr.cbits[(int64_t)it.row * pr.wp + w] &= ~mask[(int64_t)it.row * pr.wp + w];
}

int launch_sym_split_mask(const Problem& pr, const Item* items, const uint32_t* mask, Counters* ctr,
                          int64_t max_items, hipStream_t st) {
  if (max_items == 0 || mask == nullptr) return TSSPGEMM_OK;
  k_sym_split_mask<<<grid_for(max_items, 256), 256, 0, st>>>(pr, items, mask, ctr);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// ================================================================ count + scan

int64_t scan_block_sums_capacity(int64_t n) { return 2 * ((n + kScanRows - 1) / kScanRows + 1); }

// Per block of rows: popcount of each C bitmap row (nnz of the row) and the
// block totals of nnz and of products; block_sums holds nb nnz totals
// followed by nb product totals. With `bin`, also the histogram of the
// rows' numeric (class, bin) keys into the counters (num_count).
__global__ __launch_bounds__(kScanThreads) void k_count_rows(Problem pr, int32_t* cnt, int64_t* block_sums,
                                                             NumBinArgs nb, bool bin, Counters* ctr) {
  __shared__ long long sh[32];
  __shared__ int32_t hist[kNumClasses * kBins];
  if (bin) {
    for (int t = threadIdx.x; t < kNumClasses * kBins; t += blockDim.x) hist[t] = 0;
    __syncthreads();
  }
  const int64_t base = (int64_t)blockIdx.x * kScanRows;
  long long s = 0, f = 0;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    const int64_t i = base + u * kScanThreads + threadIdx.x;
    if (i < pr.n) {
      int c = 0;
      if (pr.cbits) {  // bitmap accumulator: count = popcount of the row
        const uint32_t* b = pr.cbits + i * pr.wp;
        for (int w = 0; w < pr.wp; ++w) c += __popc(b[w]);
        cnt[i] = c;
      } else {  // counts already in cnt (hash accumulator)
        c = cnt[i];
      }
      s += c;
      const int64_t fi = pr.flops[i];
      f += fi;
      if (bin && fi > 0) {
        int cls, key, count, ce;
        num_key(fi, pr.arp[i + 1] - pr.arp[i], nb.th, cls, key, count, ce);
        atomicAdd(&hist[key], count);
      }
    }
  }
  long long tot, ftot;
  block_exscan_1024(s, sh, &tot);
  block_exscan_1024(f, sh, &ftot);
  if (threadIdx.x == 0) {
    block_sums[blockIdx.x] = tot;
    block_sums[gridDim.x + blockIdx.x] = ftot;
  }
  if (bin) {
    __syncthreads();
    for (int t = threadIdx.x; t < kNumClasses * kBins; t += blockDim.x)
      if (hist[t]) atomicAdd(&(&ctr->num_count[0][0])[t], hist[t]);
  }
}

// one workgroup: exclusive scan of the block sums, nnz(C) into the counters
__global__ __launch_bounds__(kScanThreads) void k_scan_block_sums(int64_t nblocks, int64_t* block_sums,
                                                                   Counters* ctr) {
  __shared__ long long sh[32];
  long long carry = 0, fcarry = 0;
  for (int64_t b0 = 0; b0 < nblocks; b0 += kScanThreads) {
    const int64_t b = b0 + threadIdx.x;
    const long long v = b < nblocks ? block_sums[b] : 0;
    const long long f = b < nblocks ? block_sums[nblocks + b] : 0;
    long long tot, ftot;
    const long long ex = block_exscan_1024(v, sh, &tot);
    block_exscan_1024(f, sh, &ftot);
    if (b < nblocks) block_sums[b] = carry + ex;
    carry += tot;
    fcarry += ftot;
  }
  if (threadIdx.x == 0) {
    ctr->nnz_total = carry;
    ctr->flops_total = fcarry;
  }
}

// Numeric items of rows [r0, r1), one workgroup. Items are placed with one
// global reservation per (class, bin) bucket per workgroup (counts from a
// first pass over its rows): the bucket's offset (an exclusive scan of the
// bucket counts, done by every workgroup: 128 values) plus the bucket's fill
// counter (num_cursor, zero at the start); the slot inside the workgroup's
// range comes from an LDS counter in the second pass. Workgroup 0 also
// stores the class totals.
__device__ __forceinline__ void num_fill_rows(const Problem& pr, const NumBinArgs& nb, Counters* ctr, int64_t r0,
                                              int64_t r1) {
  __shared__ int32_t cnt[kNumClasses * kBins], base[kNumClasses * kBins], off[kNumClasses * kBins];
  __shared__ int32_t nsplit, split_base;
  for (int t = threadIdx.x; t < kNumClasses * kBins; t += blockDim.x) cnt[t] = 0;
  if (threadIdx.x == 0) {
    nsplit = 0;
    int32_t o = 0;
    for (int t = 0; t < kNumClasses * kBins; ++t) {
      off[t] = o;
      o += (&ctr->num_count[0][0])[t];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < kNumClasses) {
    int32_t tot = 0;
    for (int b = 0; b < kBins; ++b) tot += ctr->num_count[threadIdx.x][b];
    (&ctr->num_split_items)[threadIdx.x] = tot;  // split, block, wave, light: consecutive fields
  }
  __syncthreads();
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const int64_t f = pr.flops[i];
    if (f > 0) {
      int cls, key, count, ce;
      num_key(f, pr.arp[i + 1] - pr.arp[i], nb.th, cls, key, count, ce);
      atomicAdd(&cnt[key], count);
      if (cls == 0) atomicAdd(&nsplit, 1);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kNumClasses * kBins; t += blockDim.x) {
    if (cnt[t]) base[t] = off[t] + atomicAdd(&(&ctr->num_cursor[0][0])[t], cnt[t]);
    cnt[t] = 0;
  }
  if (threadIdx.x == 0) {
    if (nsplit) split_base = atomicAdd(&ctr->num_split_rows, nsplit);
    nsplit = 0;
  }
  __syncthreads();
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const int64_t f = pr.flops[i];
    if (f <= 0) continue;
    const int a = pr.arp[i], m = pr.arp[i + 1] - a;
    int cls, key, count, ce;
    num_key(f, m, nb.th, cls, key, count, ce);
    const int pos = base[key] + atomicAdd(&cnt[key], count);
    if (cls == 0) {
      for (int c = 0; c < count; ++c) {
        const int p0 = a + c * ce;
        nb.items[pos + c] = Item{(int32_t)i, p0, min(a + m, p0 + ce), pos + c};
      }
      nb.split_rows[split_base + atomicAdd(&nsplit, 1)] = SplitRow{(int32_t)i, pos, count, 0};
    } else {
      nb.items[pos] = Item{(int32_t)i, a, a + m, cls == 1 ? kNoSlot : 0};
    }
  }
}

// C's row pointers of the block's rows from the scanned block sums; with
// `bin`, also the block's numeric items (num_fill_rows: the bucket counts
// are complete once k_count_rows has finished).
__global__ __launch_bounds__(kScanThreads) void k_write_rowptr(Problem pr, const int32_t* cnt,
                                                               const int64_t* block_sums, int32_t* crp,
                                                               NumBinArgs nb, bool bin, Counters* ctr) {
  __shared__ long long sh[32];
  const int64_t base = (int64_t)blockIdx.x * kScanRows;
  long long carry = block_sums[blockIdx.x];
  for (int u = 0; u < kScanPer; ++u) {
    const int64_t i = base + u * kScanThreads + threadIdx.x;
    const long long v = i < pr.n ? cnt[i] : 0;
    long long tot;
    const long long ex = block_exscan_1024(v, sh, &tot);
    // int32 row pointers: the host rejects nnz(C) > INT32_MAX before use
    if (i < pr.n) crp[i] = (int32_t)(carry + ex);
    carry += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) crp[pr.n] = (int32_t)ctr->nnz_total;
  if (bin) num_fill_rows(pr, nb, ctr, base, min((int64_t)pr.n, base + kScanRows));
}

int launch_count_scan(const Problem& pr, int32_t* cnt, int64_t* block_sums, int32_t* c_rowptr, Counters* ctr,
                      hipStream_t st, const NumBinArgs* nb) {
  const int64_t nb_blocks = (pr.n + kScanRows - 1) / kScanRows;
  const NumBinArgs args = nb ? *nb : NumBinArgs{};
  const bool bin = nb != nullptr;
  if (nb_blocks > 0) k_count_rows<<<(unsigned)nb_blocks, kScanThreads, 0, st>>>(pr, cnt, block_sums, args, bin, ctr);
  k_scan_block_sums<<<1, kScanThreads, 0, st>>>(nb_blocks, block_sums, ctr);
  if (nb_blocks > 0)
    k_write_rowptr<<<(unsigned)nb_blocks, kScanThreads, 0, st>>>(pr, cnt, block_sums, c_rowptr, args, bin, ctr);
  else
    k_fill_i32<<<1, 64, 0, st>>>(c_rowptr, 1, 0);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// ================================================================ generic exclusive scan

__global__ __launch_bounds__(kScanThreads) void k_scan_sum_i32(int64_t n, const int32_t* __restrict__ in,
                                                              int64_t* __restrict__ block_sums) {
  __shared__ long long sh[32];
  const int64_t base = (int64_t)blockIdx.x * kScanRows;
  long long s = 0;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    const int64_t i = base + u * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  long long tot;
  block_exscan_1024(s, sh, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_blocks_i64(int64_t nblocks, int64_t* block_sums,
                                                                 int64_t* total) {
  __shared__ long long sh[32];
  long long carry = 0;
  for (int64_t b0 = 0; b0 < nblocks; b0 += kScanThreads) {
    const int64_t b = b0 + threadIdx.x;
    const long long v = b < nblocks ? block_sums[b] : 0;
    long long tot;
    const long long ex = block_exscan_1024(v, sh, &tot);
    if (b < nblocks) block_sums[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_write_i32(int64_t n, const int32_t* __restrict__ in,
                                                                const int64_t* __restrict__ block_sums,
                                                                int32_t* __restrict__ out) {
  __shared__ long long sh[32];
  const int64_t base = (int64_t)blockIdx.x * kScanRows;
  long long carry = block_sums[blockIdx.x];
  for (int u = 0; u < kScanPer; ++u) {
    const int64_t i = base + u * kScanThreads + threadIdx.x;
    const long long v = i < n ? in[i] : 0;
    long long tot;
    const long long ex = block_exscan_1024(v, sh, &tot);
    if (i < n) out[i] = (int32_t)(carry + ex);
    if (i == n - 1) out[n] = (int32_t)(carry + ex + v);
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sum_i64(int64_t n, const int64_t* __restrict__ in,
                                                              int64_t* __restrict__ block_sums) {
  __shared__ long long sh[32];
  const int64_t base = (int64_t)blockIdx.x * kScanRows;
  long long s = 0;
#pragma unroll
  for (int u = 0; u < kScanPer; ++u) {
    const int64_t i = base + u * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  long long tot;
  block_exscan_1024(s, sh, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_write_i64(int64_t n, const int64_t* __restrict__ in,
                                                                const int64_t* __restrict__ block_sums,
                                                                int64_t* __restrict__ out) {
  __shared__ long long sh[32];
  const int64_t base = (int64_t)blockIdx.x * kScanRows;
  long long carry = block_sums[blockIdx.x];
  for (int u = 0; u < kScanPer; ++u) {
    const int64_t i = base + u * kScanThreads + threadIdx.x;
    const long long v = i < n ? in[i] : 0;
    long long tot;
    const long long ex = block_exscan_1024(v, sh, &tot);
    if (i < n) out[i] = carry + ex;
    if (i == n - 1) out[n] = carry + ex + v;
    carry += tot;
  }
}

int64_t exscan_workspace_bytes(int64_t n) { return 8 * ((n + kScanRows - 1) / kScanRows + 1); }

// out[0..n] = exclusive prefix sums of in[0..n), int64 (out[n] = total).
int launch_exscan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* block_sums, hipStream_t st) {
  const int64_t nb = (n + kScanRows - 1) / kScanRows;
  if (nb == 0) return launch_zero_bytes(out, 8, st);
  k_scan_sum_i64<<<(unsigned)nb, kScanThreads, 0, st>>>(n, in, block_sums);
  k_scan_blocks_i64<<<1, kScanThreads, 0, st>>>(nb, block_sums, nullptr);
  k_scan_write_i64<<<(unsigned)nb, kScanThreads, 0, st>>>(n, in, block_sums, out);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// out[0..n] = exclusive prefix sums of in[0..n) (out[n] = total, int32).
int launch_exscan_i32(const int32_t* in, int64_t n, int32_t* out, int64_t* block_sums, hipStream_t st) {
  const int64_t nb = (n + kScanRows - 1) / kScanRows;
  if (nb == 0) {
    k_fill_i32<<<1, 64, 0, st>>>(out, 1, 0);
    TSS_CHECK_LAUNCH();
    return TSSPGEMM_OK;
  }
  k_scan_sum_i32<<<(unsigned)nb, kScanThreads, 0, st>>>(n, in, block_sums);
  k_scan_blocks_i64<<<1, kScanThreads, 0, st>>>(nb, block_sums, nullptr);
  k_scan_write_i32<<<(unsigned)nb, kScanThreads, 0, st>>>(n, in, block_sums, out);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

}  // namespace tss
