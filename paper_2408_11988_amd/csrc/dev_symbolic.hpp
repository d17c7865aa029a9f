// Device routines of the symbolic phase shared by the single-product and the
// batched kernels: the CSR-to-bitmap block and a 1024-thread block scan.
#pragma once

#include "core.hpp"

namespace tss {

// CSR pattern -> bitmap rows. A workgroup owns kBmRows consecutive rows
// starting at r0: it stages their row pointers and an all-zero bitmap in LDS.
// Groups of kBmLanes lanes take the rows in turn; a group streams its row's
// entries (consecutive lanes on consecutive entries, so the loads are
// coalesced and no entry has to search for its row), sets each bit with an
// LDS atomicOr, and the workgroup writes the finished bitmap rows out
// contiguously. `sm` holds kBmRows + 1 + kBmRows * wp words; blockDim.x is a
// multiple of kBmLanes. Optionally each column id is also written narrowed
// to 8 or 16 bits.
constexpr int kBmRows = 256;
constexpr int kBmLanes = 8;

__device__ __forceinline__ void bitmap_block(int64_t n, const int32_t* __restrict__ rp,
                                             const int32_t* __restrict__ ci, int wp, uint32_t* __restrict__ bits,
                                             int64_t r0, uint32_t* sm, uint8_t* __restrict__ narrow8 = nullptr,
                                             uint16_t* __restrict__ narrow16 = nullptr) {
  int32_t* srp = (int32_t*)sm;
  uint32_t* sb = sm + kBmRows + 1;
  const int nr = (int)min((int64_t)kBmRows, n - r0);
  for (int t = threadIdx.x; t <= nr; t += blockDim.x) srp[t] = rp[r0 + t];
  for (int t = threadIdx.x; t < nr * wp; t += blockDim.x) sb[t] = 0u;
  __syncthreads();
  const int grp = threadIdx.x / kBmLanes, gl = threadIdx.x % kBmLanes;
  const int ngrp = blockDim.x / kBmLanes;
  for (int r = grp; r < nr; r += ngrp) {
    uint32_t* row = sb + r * wp;
    const int q1 = srp[r + 1];
    for (int q = srp[r] + gl; q < q1; q += kBmLanes) {
      const int j = ci[q];
      atomicOr(&row[j >> 5], 1u << (j & 31));
      if (narrow8) narrow8[q] = (uint8_t)j;  // the same pass narrows the column ids
      if (narrow16) narrow16[q] = (uint16_t)j;
    }
  }
  __syncthreads();
  uint32_t* out = bits + r0 * wp;
  for (int t = threadIdx.x; t < nr * wp; t += blockDim.x) out[t] = sb[t];
}

// A bitmap row of WP words held in registers (WP <= 8), OR-ed from B's
// bitmap rows with 16-byte loads, counting the products (set bits) on the way.
template <int WP>
struct BmRow {
  uint32_t w[WP];
};

template <int WP>
__device__ __forceinline__ void bm_load_or(const uint32_t* __restrict__ src, BmRow<WP>& acc, int& fl) {
  if constexpr (WP >= 4) {
#pragma unroll
    for (int q = 0; q < WP / 4; ++q) {
      const uint4 x = reinterpret_cast<const uint4*>(src)[q];
      acc.w[4 * q] |= x.x;
      acc.w[4 * q + 1] |= x.y;
      acc.w[4 * q + 2] |= x.z;
      acc.w[4 * q + 3] |= x.w;
      fl += __popc(x.x) + __popc(x.y) + __popc(x.z) + __popc(x.w);
    }
  } else if constexpr (WP == 2) {
    const uint2 x = *reinterpret_cast<const uint2*>(src);
    acc.w[0] |= x.x;
    acc.w[1] |= x.y;
    fl += __popc(x.x) + __popc(x.y);
  } else {
    const uint32_t x = *src;
    acc.w[0] |= x;
    fl += __popc(x);
  }
}

template <int WP>
__device__ __forceinline__ void bm_store(uint32_t* __restrict__ dst, const BmRow<WP>& acc) {
  if constexpr (WP >= 4) {
#pragma unroll
    for (int q = 0; q < WP / 4; ++q)
      reinterpret_cast<uint4*>(dst)[q] = make_uint4(acc.w[4 * q], acc.w[4 * q + 1], acc.w[4 * q + 2], acc.w[4 * q + 3]);
  } else if constexpr (WP == 2) {
    *reinterpret_cast<uint2*>(dst) = make_uint2(acc.w[0], acc.w[1]);
  } else {
    *dst = acc.w[0];
  }
}


// OR of each of the WP words of `acc` over a group of G aligned lanes
// (WP <= G), reduce-scattered: at the step of lane bit o (G/2, G/4, ...) the
// lanes with that bit set keep the upper half of their words and send the
// lower half, the others the reverse, until one word is left; the remaining
// steps OR that word over the rest of the group. WP - 1 + log2(G / WP)
// shuffles in all (7 for WP = 4 over a wavefront, where a word-by-word
// reduction takes 24). Lane gl of the group ends with word
// bm_word_of<WP, G>(gl), fully reduced.
template <int WP, int G = kWave>
__device__ __forceinline__ int bm_word_of(int gl) {
  static_assert(WP <= G, "a group needs at least one lane per word");
  int w = 0;
#pragma unroll
  for (int h = WP / 2, o = G / 2; h >= 1; h >>= 1, o >>= 1)
    if (gl & o) w += h;
  return w;
}

template <int WP, int G = kWave>
__device__ __forceinline__ uint32_t bm_wave_or(const BmRow<WP>& acc, int gl) {
  static_assert(WP <= G, "a group needs at least one lane per word");
  uint32_t v[WP];
#pragma unroll
  for (int i = 0; i < WP; ++i) v[i] = acc.w[i];
  int o = G / 2;
#pragma unroll
  for (int h = WP / 2; h >= 1; h >>= 1, o >>= 1) {
    const bool hi = (gl & o) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const uint32_t send = hi ? v[i] : v[h + i];
      const uint32_t keep = hi ? v[h + i] : v[i];
      v[i] = keep | shfl_xor_u32(send, o);
    }
  }
  for (; o >= 1; o >>= 1) v[0] |= shfl_xor_u32(v[0], o);
  return v[0];
}

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanRows = kScanThreads * kScanPer;


// exclusive scan of v over the 1024 threads of the block; returns the prefix,
// total in *tot. Uses a 16-entry shared array.
__device__ __forceinline__ long long block_exscan_1024(long long v, long long* sh, long long* tot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  long long x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    long long y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  if (wave == 0) {
    long long s = lane < 16 ? sh[lane] : 0;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      long long y = __shfl_up(s, o, kWave);
      if (lane >= o) s += y;
    }
    if (lane < 16) sh[16 + lane] = s;  // inclusive prefix of wave totals
  }
  __syncthreads();
  const long long before = wave ? sh[16 + wave - 1] : 0;
  *tot = sh[16 + 15];
  __syncthreads();
  return before + x - v;
}



// Work class of a row with m > 0 entries: floor(log2 m) mapped so that heavier
// rows get smaller bin numbers; bin 0 holds the chunks of split rows.
__device__ __forceinline__ int bin_of(int64_t work) {
  const int e = 63 - __clzll((unsigned long long)work);
  const int b = kBins - 1 - e;
  return b < 1 ? 1 : b;
}

// bin and item count of row i in the heavy-row list (count 0: not listed)
__device__ __forceinline__ void sym_bin(int m, int32_t split_nnz, int& bin, int& count,
                                        int light_max = kSlotRowMax) {
  if (m <= light_max) {
    bin = 0;
    count = 0;
  } else if (m <= split_nnz) {
    bin = bin_of(m);
    count = 1;
  } else {
    bin = 0;
    count = (m + split_nnz - 1) / split_nnz;
  }
}

// Columns < d in bitmap word w (all ones for a whole word, none past d).
__device__ __forceinline__ uint32_t word_cols(int d, int w) {
  const int wb = 32 * w;
  return d >= wb + 32 ? 0xffffffffu : (d > wb ? (1u << (d - wb)) - 1u : 0u);
}

// One heavy item's pattern over a wavefront, a lane per A entry: the OR of
// the B bitmap rows of A entries [p0, p1), returned reduce-scattered (this
// lane's word bm_word_of<WP>(lane), OR-ed over the wavefront); the products
// (the B rows' lengths) are added to fl, per lane. Whole rounds of 2 * 64
// entries, each followed by a check: once the accumulator holds every column
// < d no later B row can change the pattern, and the rest of the item only
// adds its B rows' lengths, read from B's row pointers instead of gathering
// their bitmaps (in R-MAT rows a hub's pattern fills after a few dozen B
// rows). B's columns are strictly increasing, so a bitmap row's popcount is
// its length.
template <int WP>
__device__ __forceinline__ uint32_t sym_item_or(const Problem& pr, int p0, int p1, int lane, int& fl) {
  const uint32_t* __restrict__ bb = pr.bbits;
  const int32_t* __restrict__ aci = pr.aci;
  const uint32_t wfull = word_cols(pr.d, bm_word_of<WP>(lane));
  BmRow<WP> acc;
#pragma unroll
  for (int w = 0; w < WP; ++w) acc.w[w] = 0u;
  uint32_t word = 0u;
  bool full = false;
  int p = p0;
  for (; p + 2 * kWave <= p1; p += 2 * kWave) {  // wavefront-uniform rounds
    const int k0 = aci[p + lane], k1 = aci[p + kWave + lane];
    bm_load_or<WP>(bb + (int64_t)k0 * WP, acc, fl);
    bm_load_or<WP>(bb + (int64_t)k1 * WP, acc, fl);
    word = bm_wave_or<WP>(acc, lane);
    if (__ballot(word != wfull) == 0ull) {
      full = true;
      p += 2 * kWave;
      break;
    }
  }
  p += lane;
  if (full) {
    const int32_t* __restrict__ brp = pr.brp;
    for (; p + 3 * kWave < p1; p += 4 * kWave) {
      const int k0 = aci[p], k1 = aci[p + kWave], k2 = aci[p + 2 * kWave], k3 = aci[p + 3 * kWave];
      fl += (brp[k0 + 1] - brp[k0]) + (brp[k1 + 1] - brp[k1]) + (brp[k2 + 1] - brp[k2]) + (brp[k3 + 1] - brp[k3]);
    }
    for (; p < p1; p += kWave) {
      const int k = aci[p];
      fl += brp[k + 1] - brp[k];
    }
    return word;
  }
  for (; p < p1; p += kWave) bm_load_or<WP>(bb + (int64_t)aci[p] * WP, acc, fl);
  return bm_wave_or<WP>(acc, lane);
}

// One heavy item's pattern in slots of wp lanes (a lane per bitmap word,
// 64 / wp B rows in flight): lane (slot, w) ORs word w of the B rows of
// entries p0 + slot, p0 + slot + ns, ... and returns it (not yet OR-ed over
// the slots); its popcounts are added to fl. Whole rounds of 4 * ns entries,
// each followed by a check: once the accumulator, OR-ed over the slots, holds
// every column of `need` (this lane's word: the columns the result can still
// gain), the rest of the item only adds its B rows' lengths (B's row
// pointers, counted by the slot's word-0 lane) without gathering bitmaps.
__device__ __forceinline__ uint32_t sym_item_or_slots(const Problem& pr, int p0, int p1, int wp, int lane,
                                                      uint32_t need, int& fl) {
  const int ns = kWave / wp, slot = lane / wp, w = lane & (wp - 1);
  const uint32_t* __restrict__ bb = pr.bbits;
  const int32_t* __restrict__ aci = pr.aci;
  uint32_t acc = 0u;
  bool full = false;
  int p = p0;
  for (; p + 4 * ns <= p1; p += 4 * ns) {  // wavefront-uniform rounds
    const int q = p + slot;
    const int k0 = aci[q], k1 = aci[q + ns], k2 = aci[q + 2 * ns], k3 = aci[q + 3 * ns];
    const uint32_t x0 = bb[(int64_t)k0 * wp + w], x1 = bb[(int64_t)k1 * wp + w];
    const uint32_t x2 = bb[(int64_t)k2 * wp + w], x3 = bb[(int64_t)k3 * wp + w];
    acc |= (x0 | x1) | (x2 | x3);
    fl += __popc(x0) + __popc(x1) + __popc(x2) + __popc(x3);
    uint32_t all = acc;
    for (int o = wp; o < kWave; o <<= 1) all |= shfl_xor_u32(all, o);
    if (__ballot((need & ~all) != 0u) == 0ull) {
      full = true;
      p += 4 * ns;
      break;
    }
  }
  p += slot;
  if (full) {
    if (w == 0) {
      const int32_t* __restrict__ brp = pr.brp;
      for (; p < p1; p += ns) {
        const int k = aci[p];
        fl += brp[k + 1] - brp[k];
      }
    }
    return acc;
  }
  for (; p < p1; p += ns) {
    const uint32_t x = bb[(int64_t)aci[p] * wp + w];
    acc |= x;
    fl += __popc(x);
  }
  return acc;
}

}  // namespace tss
