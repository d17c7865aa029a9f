// Hash accumulator for wide outputs (Sec. III-C: past d = 1024 the dense
// accumulator no longer fits the nearest cache level and a hash table is used
// instead).
//
// Both phases give one wavefront to a row and walk the row's products as one
// flat list: 64 A entries are staged at a time (their B row start, length and
// value), an inclusive scan of the lengths lets lane t find its product by a
// binary search over the staged prefix sums, so every lane has work however
// short the B rows are.
//
// Symbolic: the distinct columns of the row (minus masked ones) are counted
// in an LDS open-addressing set (linear probing, column as key) of a power of
// two >= 2 min(d, flops_i) slots, or, when that exceeds the table, in an LDS
// bitmap of d bits.
// Numeric: rows with at most kHashNumMax outputs accumulate in an LDS table of
// (column, sum) slots sized from the exact output count; the table is sorted
// by key in place (bitonic, in LDS; empty slots sort last) and its first
// nnz_i slots are the row, in ascending columns. Longer rows
// mark an LDS bitmap and add into a private d-wide strip in global memory;
// the row is written by walking the bitmap (ascending columns) and the strip
// is cleared behind it.
// Masked columns are tested per product (binary search in the mask row, or a
// bit test), so tables only ever hold output columns.
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

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// ---------------------------------------------------------------- symbolic

__global__ __launch_bounds__(kHashWaves * kWave) void k_hash_symbolic(Problem pr, HashMask hm, int32_t* cnt,
                                                                      int32_t* err) {
  __shared__ uint32_t sm[kHashWaves][kSymSlots];
  __shared__ int start_s[kHashWaves][kWave], pref_s[kHashWaves][kWave + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  uint32_t* tab = sm[wave];
  int* start = start_s[wave];
  int* pref = pref_s[wave];
  const bool masked = hm.rp || hm.bits;
  for (int64_t row = (int64_t)blockIdx.x * kHashWaves + wave; row < pr.n; row += (int64_t)gridDim.x * kHashWaves) {
    const int p0 = pr.arp[row], p1 = pr.arp[row + 1];
    long long fl = 0;
    for (int p = p0 + lane; p < p1; p += kWave) {
      const int k = pr.aci[p];
      fl += pr.brp[k + 1] - pr.brp[k];
    }
    fl = wave_sum_ll(fl);
    if (lane == 0) pr.flops[row] = fl;
    if (fl == 0) {
      if (lane == 0) cnt[row] = 0;
      continue;
    }
    const int64_t ub = fl < pr.d ? fl : pr.d;
    const bool table = 2 * ub <= kSymSlots;
    const uint32_t tsz = table ? pow2_at_least((uint32_t)(2 * ub)) : 0u;
    const int words = table ? (int)tsz : (pr.d + 31) >> 5;
    for (int t = lane; t < words; t += kWave) tab[t] = table ? kEmpty : 0u;
    wave_sync();
    int fresh = 0;
    for (int base = p0; base < p1; base += kWave) {
      const int nb = min(kWave, p1 - base);
      const int total = stage_products<char>(pr, base, nb, start, pref, nullptr);
      for (int t = lane; t < total; t += kWave) {
        const int e = staged_entry(pref, t);
        const int32_t j = pr.bci[start[e] + (t - pref[e])];
        if (masked && is_masked(hm, row, j)) continue;
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
      }
      wave_sync();
    }
    const long long c = wave_sum_ll(fresh);
    if (lane == 0) cnt[row] = (int32_t)c;
    wave_sync();
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

template <typename V>
__global__ __launch_bounds__(kHashWaves * kWave) void k_hash_numeric_table(Problem pr, HashMask hm, int32_t* err) {
  using Acc = typename HashAcc<V>::type;
  __shared__ uint32_t keys_s[kHashWaves][kNumSlots];
  __shared__ Acc vals_s[kHashWaves][kNumSlots];
  __shared__ int start_s[kHashWaves][kWave], pref_s[kHashWaves][kWave + 1];
  __shared__ V aval_s[kHashWaves][kWave];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  uint32_t* keys = keys_s[wave];
  Acc* vals = vals_s[wave];
  const bool masked = hm.rp || hm.bits;
  const V* __restrict__ bval = (const V*)pr.bval;
  for (int64_t row = (int64_t)blockIdx.x * kHashWaves + wave; row < pr.n; row += (int64_t)gridDim.x * kHashWaves) {
    const int c0 = pr.crp[row], nnz = pr.crp[row + 1] - c0;
    if (nnz == 0 || nnz > kHashNumMax) continue;
    const uint32_t tsz = pow2_at_least(2u * (uint32_t)nnz);  // <= kNumSlots
    for (uint32_t t = lane; t < tsz; t += kWave) {
      keys[t] = kEmpty;
      vals[t] = Acc(0);
    }
    wave_sync();
    const int p0 = pr.arp[row], p1 = pr.arp[row + 1];
    for (int base = p0; base < p1; base += kWave) {
      const int nb = min(kWave, p1 - base);
      const int total = stage_products<V>(pr, base, nb, start_s[wave], pref_s[wave], aval_s[wave]);
      for (int t = lane; t < total; t += kWave) {
        const int e = staged_entry(pref_s[wave], t);
        const int q = start_s[wave][e] + (t - pref_s[wave][e]);
        const int32_t j = pr.bci[q];
        if (masked && is_masked(hm, row, j)) continue;
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
          if (h != kEmpty) lds_add(&vals[h], hash_prod<V>(aval_s[wave][e], bval[q]));
      }
      wave_sync();
    }
    // sort the whole table by key: empty slots (all ones) go last, the row's
    // nnz columns come first in ascending order
    wave_bitonic<Acc>(keys, vals, (int)tsz);
    for (int t = lane; t < nnz; t += kWave) {
      pr.cci[c0 + t] = (int32_t)keys[t];
      if constexpr (!std::is_same<V, char>::value) ((V*)pr.cval)[c0 + t] = SemiringT<V>::out(vals[t]);
    }
    if (lane == 0 && (keys[nnz - 1] == kEmpty || ((uint32_t)nnz < tsz && keys[nnz] != kEmpty))) atomicOr(err, 1);
    wave_sync();
  }
}

// Rows with more than kHashNumMax outputs: LDS bitmap of d bits, private
// d-wide strip in global memory (kept all-zero between rows).
template <typename V>
__global__ __launch_bounds__(kHashWaves * kWave) void k_hash_numeric_dense(Problem pr, HashMask hm,
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
  const V* __restrict__ bval = (const V*)pr.bval;
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
    if (nnz <= kHashNumMax) continue;
    const int64_t row_id = r;
    const int p0 = pr.arp[row_id], p1 = pr.arp[row_id + 1];
    for (int base = p0; base < p1; base += kWave) {
      const int nb = min(kWave, p1 - base);
      const int total = stage_products<V>(pr, base, nb, start_s[wave], pref_s[wave], aval_s[wave]);
      for (int t = lane; t < total; t += kWave) {
        const int e = staged_entry(pref_s[wave], t);
        const int q = start_s[wave][e] + (t - pref_s[wave][e]);
        const int32_t j = pr.bci[q];
        if (masked && is_masked(hm, row_id, j)) continue;
        atomicOr(&bm[j >> 5], 1u << (j & 31));
        if constexpr (!std::is_same<V, char>::value) {
          if constexpr (sizeof(Acc) == 8)
            atomicAdd(&strip[j], hash_prod<V>(aval_s[wave][e], bval[q]));
          else
            atomicAdd((unsigned int*)&strip[j], (unsigned int)hash_prod<V>(aval_s[wave][e], bval[q]));
        }
      }
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

// ---------------------------------------------------------------- launch

// One wavefront per row (no grid stride), so the hardware's workgroup
// dispatch balances rows of very different lengths.
int launch_hash_symbolic(const Problem& pr, const HashMask& m, int32_t* cnt, int32_t* err, hipStream_t st) {
  if (pr.n == 0) return TSSPGEMM_OK;
  const int64_t g = (pr.n + kHashWaves - 1) / kHashWaves;
  k_hash_symbolic<<<(unsigned)g, kHashWaves * kWave, 0, st>>>(pr, m, cnt, err);
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

int launch_hash_numeric(int sr, const Problem& pr, const HashMask& h, void* strips, int32_t* err, int32_t* next,
                        hipStream_t st) {
  if (pr.n == 0) return TSSPGEMM_OK;
  const int64_t g = (pr.n + kHashWaves - 1) / kHashWaves;  // table rows: one wavefront per row
  int64_t gd = hash_dense_workers(pr.d) / kHashWaves;
  if (gd > g) gd = g;
  int rc;
  if ((rc = launch_zero_bytes(next, 4, st))) return rc;
  if (sr == TSSPGEMM_PLUS_TIMES_F32) {
    k_hash_numeric_table<float><<<(unsigned)g, kHashWaves * kWave, 0, st>>>(pr, h, err);
    k_hash_numeric_dense<float><<<(unsigned)gd, kHashWaves * kWave, 0, st>>>(pr, h, (double*)strips, err, next);
  } else if (sr == TSSPGEMM_PLUS_TIMES_I32) {
    k_hash_numeric_table<int32_t><<<(unsigned)g, kHashWaves * kWave, 0, st>>>(pr, h, err);
    k_hash_numeric_dense<int32_t><<<(unsigned)gd, kHashWaves * kWave, 0, st>>>(pr, h, (int32_t*)strips, err, next);
  } else {
    k_hash_numeric_table<char><<<(unsigned)g, kHashWaves * kWave, 0, st>>>(pr, h, err);
    k_hash_numeric_dense<char><<<(unsigned)gd, kHashWaves * kWave, 0, st>>>(pr, h, (int32_t*)strips, err, next);
  }
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

}  // namespace tss
