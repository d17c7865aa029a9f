// Device routines of the numeric phase shared by the single-product and the
// batched kernels: semiring arithmetic, LDS strip accumulation of one A row
// (or a range of its entries), and the compaction of a strip into C's row.
#pragma once

#include "core.hpp"

namespace tss {

template <typename T>
struct SemiringT;
template <>
struct SemiringT<float> {  // plus-times over FP32 inputs, FP64 accumulation
  using acc = double;
  __device__ static acc prod(float a, float b) { return (double)a * (double)b; }
  __device__ static float out(acc x) { return (float)x; }
  __device__ static acc add(acc x, acc y) { return x + y; }
};
template <>
struct SemiringT<int32_t> {  // plus-times over int32, wrap-around
  using acc = int32_t;
  __device__ static acc prod(int32_t a, int32_t b) { return (int32_t)((uint32_t)a * (uint32_t)b); }
  __device__ static int32_t out(acc x) { return x; }
  __device__ static acc add(acc x, acc y) { return (int32_t)((uint32_t)x + (uint32_t)y); }
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void lds_add(double* p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void lds_add(int32_t* p, int32_t v) { atomicAdd((unsigned int*)p, (unsigned int)v); }

constexpr int kHeavyUnroll = 4;  // A entries per group per step, wavefront / workgroup rows
constexpr int kLightUnroll = 4;  // A entries per group per step, light rows

// ---------------------------------------------------------------- wavefront / workgroup rows

// B column ids as IdxT: int32_t reads B's own array, uint8_t / uint16_t the
// narrowed copy (fewer bytes per gathered B row).
template <typename IdxT>
__device__ __forceinline__ const IdxT* col_ids(const Problem& pr) {
  if constexpr (sizeof(IdxT) == 4)
    return (const IdxT*)pr.bci;
  else
    return (const IdxT*)pr.bcol;
}

// Accumulate entries [p_begin, p_end) of one A row into `strip`, taking
// 64-entry batches number wstart, wstart + wstride, ... (one wavefront): the
// batch is staged (entry, B row bounds, value) through LDS, and the 64/GL
// groups of the wavefront each take a B row, GL entries per step, U rows per
// group in flight ("per B row" product layout).
template <int GL, typename T, typename IdxT = int32_t>
__device__ __forceinline__ void accumulate_range_rows(const Problem& pr, int p_begin, int p_end, int wstart, int wstride,
                                                 typename SemiringT<T>::acc* strip, int4* stage) {
  using S = SemiringT<T>;
  constexpr int GPW = kWave / GL;
  constexpr int U = kHeavyUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  const int grp = lane / GL, gl = lane % GL;
  const int32_t* __restrict__ aci = pr.aci;
  const T* __restrict__ aval = (const T*)pr.aval;
  const int32_t* __restrict__ brp = pr.brp;
  const IdxT* __restrict__ bci = col_ids<IdxT>(pr);
  const T* __restrict__ bval = (const T*)pr.bval;

  for (int base = p_begin + kWave * wstart; base < p_end; base += kWave * wstride) {
    const int nb = min(kWave, p_end - base);
    int4 e = make_int4(0, 0, 0, 0);
    if (lane < nb) {
      const int k = aci[base + lane];
      T a = aval[base + lane];
      e.x = brp[k];
      e.y = brp[k + 1];
      e.z = __builtin_bit_cast(int32_t, a);
    }
    wave_sync();
    stage[lane] = e;
    wave_sync();
    for (int s = 0; s < nb; s += U * GPW) {
      int q[U], qe[U];
      int jj[U];
      T av[U], bv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = s + u * GPW + grp;
        int4 r = make_int4(0, 0, 0, 0);
        if (src < nb) r = stage[src];
        q[u] = r.x + gl;
        qe[u] = r.y;
        av[u] = __builtin_bit_cast(T, r.z);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] < qe[u]) {
          jj[u] = bci[q[u]];
          bv[u] = bval[q[u]];
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] < qe[u]) lds_add(&strip[jj[u]], S::prod(av[u], bv[u]));
#pragma unroll
      for (int u = 0; u < U; ++u)
        for (int qq = q[u] + GL; qq < qe[u]; qq += GL) lds_add(&strip[bci[qq]], S::prod(av[u], bval[qq]));
    }
    wave_sync();
  }
}

// Accumulate entries [p_begin, p_end) of one A row into `strip`, taking
// 64-entry batches number wstart, wstart + wstride, ... (one wavefront). A
// batch is staged as in accumulate_light, with the whole wavefront as the
// group: lane t loads entry t and its B row bounds (coalesced), a wavefront
// scan of the B row lengths makes the batch's products one flat list, and
// lane t takes products t, t + 64, ... (U per step, independent loads).
template <typename T, typename IdxT = int32_t>
__device__ __forceinline__ void accumulate_range_flat(const Problem& pr, int p_begin, int p_end, int wstart, int wstride,
                                                 typename SemiringT<T>::acc* strip, int4* stage) {
  using S = SemiringT<T>;
  constexpr int U = kHeavyUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t* __restrict__ aci = pr.aci;
  const T* __restrict__ aval = (const T*)pr.aval;
  const int32_t* __restrict__ brp = pr.brp;
  const IdxT* __restrict__ bci = col_ids<IdxT>(pr);
  const T* __restrict__ bval = (const T*)pr.bval;

  for (int base = p_begin + kWave * wstart; base < p_end; base += kWave * wstride) {
    const int nb = min(kWave, p_end - base);
    int q0 = 0, len = 0;
    T a = T(0);
    if (lane < nb) {
      const int k = aci[base + lane];
      a = aval[base + lane];
      q0 = brp[k];
      len = brp[k + 1] - q0;
    }
    int incl = len;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    const int total = __shfl(incl, kWave - 1, kWave);
    wave_sync();
    stage[lane] = make_int4(q0 - (incl - len), incl, __builtin_bit_cast(int32_t, a), 0);
    wave_sync();
    int e = 0;
    int4 cur = stage[0];
    for (int f0 = 0; f0 < total; f0 += U * kWave) {
      int q[U];
      T av[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int f = f0 + u * kWave + lane;
        q[u] = -1;
        av[u] = T(0);
        if (f < total) {
          while (cur.y <= f) cur = stage[++e];
          q[u] = cur.x + f;
          av[u] = __builtin_bit_cast(T, cur.z);
        }
      }
      int jj[U];
      T bv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        jj[u] = 0;
        bv[u] = T(0);
        if (q[u] >= 0) {
          jj[u] = bci[q[u]];
          bv[u] = bval[q[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] >= 0) lds_add(&strip[jj[u]], S::prod(av[u], bv[u]));
    }
    wave_sync();
  }
}

// Product layout of a wavefront's batch: per B row (FLAT false) or flat.
template <int GL, typename T, typename IdxT, bool FLAT>
__device__ __forceinline__ void accumulate_range(const Problem& pr, int p_begin, int p_end, int wstart, int wstride,
                                                 typename SemiringT<T>::acc* strip, int4* stage) {
  if constexpr (FLAT)
    accumulate_range_flat<T, IdxT>(pr, p_begin, p_end, wstart, wstride, strip, stage);
  else
    accumulate_range_rows<GL, T, IdxT>(pr, p_begin, p_end, wstart, wstride, strip, stage);
}

// Write row `row` of C from a strip: wavefront `wave_id` of `nwaves` handles
// 64-column chunks wave_id, wave_id + nwaves, ...
template <typename T>
__device__ __forceinline__ void emit_row(const Problem& pr, int64_t row, const typename SemiringT<T>::acc* strip,
                                         int wave_id, int nwaves) {
  using S = SemiringT<T>;
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t* cb = pr.cbits + row * pr.wp;
  const int nch = (pr.d + 63) >> 6;
  int base = pr.crp[row];
  for (int w = 0; w < 2 * wave_id && w < pr.wp; ++w) base += __popc(cb[w]);
  for (int c = wave_id; c < nch; c += nwaves) {
    const uint32_t lo = cb[2 * c];
    const uint32_t hi = (2 * c + 1 < pr.wp) ? cb[2 * c + 1] : 0u;
    const uint64_t m = (uint64_t)lo | ((uint64_t)hi << 32);
    if ((m >> lane) & 1ull) {
      const int pos = base + lanes_below(m);
      const int j = 64 * c + lane;
      pr.cci[pos] = j;
      ((T*)pr.cval)[pos] = S::out(strip[j]);
    }
    for (int w = 2 * c; w < 2 * (c + nwaves) && w < pr.wp; ++w) base += __popc(cb[w]);
  }
}


// ---------------------------------------------------------------- light rows

// Write row `row` from a group's strip; the group's GL lanes handle GL-column
// chunks in order (GL <= 64, a power of two, so a chunk never straddles a
// 64-bit pair of bitmap words).
template <int GL, typename T>
__device__ __forceinline__ void emit_group(const Problem& pr, int64_t row, const typename SemiringT<T>::acc* strip,
                                           int gl) {
  using S = SemiringT<T>;
  const uint32_t* cb = pr.cbits + row * pr.wp;
  int base = pr.crp[row];
  const uint64_t below = (gl == 0) ? 0ull : ((~0ull) >> (64 - gl));
  for (int c0 = 0; c0 < pr.d; c0 += GL) {
    uint64_t m;
    if constexpr (GL == 64) {
      const int w = c0 >> 5;
      m = (uint64_t)cb[w] | ((w + 1 < pr.wp) ? ((uint64_t)cb[w + 1] << 32) : 0ull);
    } else {
      m = ((uint64_t)cb[c0 >> 5] >> (c0 & 31)) & ((1ull << GL) - 1ull);
    }
    if ((m >> gl) & 1ull) {
      const int pos = base + __popcll(m & below);
      const int j = c0 + gl;
      pr.cci[pos] = j;
      ((T*)pr.cval)[pos] = S::out(strip[j]);
    }
    base += __popcll(m);
  }
}

// Accumulate entries [p0, p1) of one A row into a group's strip (GL lanes,
// lane gl), per B row: the group stages up to GL A entries with their B row
// bounds, then takes U staged B rows per step, GL entries of each at a time.
template <int GL, typename T, typename IdxT = int32_t>
__device__ __forceinline__ void accumulate_light_rows(const Problem& pr, int p0, int p1,
                                                 typename SemiringT<T>::acc* strip, int4* stage, int gl) {
  using S = SemiringT<T>;
  constexpr int U = kLightUnroll;
  const int32_t* __restrict__ aci = pr.aci;
  const T* __restrict__ aval = (const T*)pr.aval;
  const int32_t* __restrict__ brp = pr.brp;
  const IdxT* __restrict__ bci = col_ids<IdxT>(pr);
  const T* __restrict__ bval = (const T*)pr.bval;
  for (int base = p0; base < p1; base += GL) {
    const int nb = min(GL, p1 - base);
    int4 e = make_int4(0, 0, 0, 0);
    if (gl < nb) {
      const int k = aci[base + gl];
      e.x = brp[k];
      e.y = brp[k + 1];
      e.z = __builtin_bit_cast(int32_t, aval[base + gl]);
    }
    wave_sync();
    stage[gl] = e;
    wave_sync();
    for (int s = 0; s < nb; s += U) {
      int q[U], qe[U];
      int jj[U];
      T av[U], bv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int4 r = make_int4(0, 0, 0, 0);
        if (s + u < nb) r = stage[s + u];
        q[u] = r.x + gl;
        qe[u] = r.y;
        av[u] = __builtin_bit_cast(T, r.z);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] < qe[u]) {
          jj[u] = bci[q[u]];
          bv[u] = bval[q[u]];
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] < qe[u]) lds_add(&strip[jj[u]], S::prod(av[u], bv[u]));
#pragma unroll
      for (int u = 0; u < U; ++u)
        for (int qq = q[u] + GL; qq < qe[u]; qq += GL) lds_add(&strip[bci[qq]], S::prod(av[u], bval[qq]));
    }
    wave_sync();
  }
}

// Accumulate entries [p0, p1) of one A row into a group's strip (GL lanes,
// lane gl). The group loads up to GL of the row's A entries at once, one per
// lane (coalesced), with their B row bounds, and a scan over the group turns
// the B row lengths into offsets: the products of the staged entries form one
// flat list, and lane gl takes products gl, gl + GL, ... (U of them per step,
// all loads independent). A lane finds the staged entry of its product by
// moving forward through the offsets (its product index only grows), so short
// B rows do not leave lanes idle and a step has one dependent gather.
// stage[e] = (start of B row - offset of e, end offset of e, A value bits).
template <int GL, typename T, typename IdxT = int32_t>
__device__ __forceinline__ void accumulate_light_flat(const Problem& pr, int p0, int p1,
                                                 typename SemiringT<T>::acc* strip, int4* stage, int gl) {
  using S = SemiringT<T>;
  constexpr int U = kLightUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  const int32_t* __restrict__ aci = pr.aci;
  const T* __restrict__ aval = (const T*)pr.aval;
  const int32_t* __restrict__ brp = pr.brp;
  const IdxT* __restrict__ bci = col_ids<IdxT>(pr);
  const T* __restrict__ bval = (const T*)pr.bval;
  for (int base = p0; base < p1; base += GL) {
    const int nb = min(GL, p1 - base);
    int q0 = 0, len = 0;
    T a = T(0);
    if (gl < nb) {
      const int k = aci[base + gl];
      a = aval[base + gl];
      q0 = brp[k];
      len = brp[k + 1] - q0;
    }
    int incl = len;  // inclusive scan of the lengths over the group
#pragma unroll
    for (int o = 1; o < GL; o <<= 1) {
      const int y = __shfl_up(incl, o, kWave);
      if (gl >= o) incl += y;
    }
    const int total = __shfl(incl, (lane & ~(GL - 1)) + GL - 1, kWave);
    wave_sync();
    stage[gl] = make_int4(q0 - (incl - len), incl, __builtin_bit_cast(int32_t, a), 0);
    wave_sync();
    int e = 0;
    int4 cur = stage[0];
    for (int f0 = 0; f0 < total; f0 += U * GL) {
      int q[U];
      T av[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int f = f0 + u * GL + gl;
        q[u] = -1;
        av[u] = T(0);
        if (f < total) {
          while (cur.y <= f) cur = stage[++e];
          q[u] = cur.x + f;
          av[u] = __builtin_bit_cast(T, cur.z);
        }
      }
      int jj[U];
      T bv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        jj[u] = 0;
        bv[u] = T(0);
        if (q[u] >= 0) {
          jj[u] = bci[q[u]];
          bv[u] = bval[q[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] >= 0) lds_add(&strip[jj[u]], S::prod(av[u], bv[u]));
    }
    wave_sync();
  }
}

// Product layout of a lane group's row: per B row (FLAT false) or flat.
template <int GL, typename T, typename IdxT, bool FLAT>
__device__ __forceinline__ void accumulate_light(const Problem& pr, int p0, int p1,
                                                 typename SemiringT<T>::acc* strip, int4* stage, int gl) {
  if constexpr (FLAT)
    accumulate_light_flat<GL, T, IdxT>(pr, p0, p1, strip, stage, gl);
  else
    accumulate_light_rows<GL, T, IdxT>(pr, p0, p1, strip, stage, gl);
}

// ================================================================ binning (numeric)

// Work class by a row's work: 3 = light (a lane group), 2 = one wavefront,
// 1 = one workgroup, 0 = split into chunks of at least kMinChunk A entries.
// The work is the product count, but at least kEntryWork per A entry: each
// entry is staged (its column, B row bounds and value) whether or not its B
// row holds anything, so a hub row over near-empty B rows is a long serial
// walk for one wavefront though it has few products.
constexpr int kMinChunk = 64;
constexpr int64_t kEntryWork = 16;
__device__ __forceinline__ int64_t num_work(int64_t f, int m) {
  return f > kEntryWork * m ? f : kEntryWork * m;
}

__device__ __forceinline__ int num_class(int64_t f, const NumThresholds& th) {
  return f <= th.light_max ? 3 : (f <= th.wave_max ? 2 : (f <= th.split ? 1 : 0));
}
__device__ __forceinline__ int num_bin(int64_t work) {
  const int e = 63 - __clzll((unsigned long long)work);
  const int b = kBins - 1 - e;
  return b < 0 ? 0 : b;
}
__device__ __forceinline__ int chunk_entries(int m, int64_t f, int64_t split) {
  const int64_t want = (f + split - 1) / split;  // chunks by work (num_work)
  int ce = (int)((m + want - 1) / want);
  return ce < kMinChunk ? kMinChunk : ce;
}

// (class, bin) key of a row with f > 0 products and m A entries (by its
// work, num_work), and the number of items it makes (split rows: one per
// chunk).
__device__ __forceinline__ void num_key(int64_t f, int m, const NumThresholds& th, int& cls, int& key, int& count,
                                        int& ce) {
  const int64_t w = num_work(f, m);
  cls = num_class(w, th);
  if (cls == 0) {
    ce = chunk_entries(m, w, th.split);
    count = (m + ce - 1) / ce;
    key = 0;
  } else {
    ce = 0;
    count = 1;
    key = cls * kBins + num_bin(w);
  }
}

}  // namespace tss
