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

// Readers of B's entries by their position q in B's arrays.
// BSep: column ids (narrowed to IdxT) and values from two arrays.
template <typename IdxT>
struct BSep {
  using Idx = IdxT;
  const IdxT* __restrict__ ci;
  const void* __restrict__ v;
  __device__ explicit BSep(const Problem& pr) : ci(col_ids<IdxT>(pr)), v(pr.bval) {}
  __device__ int id(int q) const { return (int)ci[q]; }
  template <typename T>
  __device__ T val(int q) const {
    return ((const T*)v)[q];
  }
};


// B row bounds (brp[k], brp[k+1]) of A entry p = (i, k): from the plan's
// per-entry record when there is one (no dependent gather), else through
// A's column, recorded when the plan asks for it.
__device__ __forceinline__ int2 entry_bounds(const Problem& pr, int p) {
  if (pr.ebnd) return pr.ebnd[p];
  const int k = pr.aci[p];
  const int2 b = make_int2(pr.brp[k], pr.brp[k + 1]);
  if (pr.ebnd_w) pr.ebnd_w[p] = b;
  return b;
}

// Accumulate entries [p_begin, p_end) of one A row into `strip`, taking
// 64-entry batches number wstart, wstart + wstride, ... (one wavefront): the
// batch is staged (entry, B row bounds, value) through LDS, and the 64/GL
// groups of the wavefront each take a B row, GL entries per step, U rows per
// group in flight ("per B row" product layout).
template <int GL, typename T, typename BR>
__device__ __forceinline__ void accumulate_range_rows(const Problem& pr, int p_begin, int p_end, int wstart, int wstride,
                                                 typename SemiringT<T>::acc* strip, int4* stage) {
  using S = SemiringT<T>;
  constexpr int GPW = kWave / GL;
  constexpr int U = kHeavyUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  const int grp = lane / GL, gl = lane % GL;
  const T* __restrict__ aval = (const T*)pr.aval;
  const BR br(pr);

  for (int base = p_begin + kWave * wstart; base < p_end; base += kWave * wstride) {
    const int nb = min(kWave, p_end - base);
    int4 e = make_int4(0, 0, 0, 0);
    if (lane < nb) {
      const int2 bnd = entry_bounds(pr, base + lane);
      T a = aval[base + lane];
      e.x = bnd.x;
      e.y = bnd.y;
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
          jj[u] = br.id(q[u]);
          bv[u] = br.template val<T>(q[u]);
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] < qe[u]) lds_add(&strip[jj[u]], S::prod(av[u], bv[u]));
#pragma unroll
      for (int u = 0; u < U; ++u)
        for (int qq = q[u] + GL; qq < qe[u]; qq += GL) lds_add(&strip[br.id(qq)], S::prod(av[u], br.template val<T>(qq)));
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
template <typename T, typename BR>
__device__ __forceinline__ void accumulate_range_flat(const Problem& pr, int p_begin, int p_end, int wstart, int wstride,
                                                 typename SemiringT<T>::acc* strip, int4* stage) {
  using S = SemiringT<T>;
  constexpr int U = kHeavyUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  const T* __restrict__ aval = (const T*)pr.aval;
  const BR br(pr);

  for (int base = p_begin + kWave * wstart; base < p_end; base += kWave * wstride) {
    const int nb = min(kWave, p_end - base);
    int q0 = 0, len = 0;
    T a = T(0);
    if (lane < nb) {
      const int2 bnd = entry_bounds(pr, base + lane);
      a = aval[base + lane];
      q0 = bnd.x;
      len = bnd.y - q0;
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
          jj[u] = br.id(q[u]);
          bv[u] = br.template val<T>(q[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] >= 0) lds_add(&strip[jj[u]], S::prod(av[u], bv[u]));
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------- 4-entry chunks of B rows

// Product layouts (template argument LAYOUT of the numeric kernels).
constexpr int kLayoutRows = 0;  // a group of GL lanes per B row, one entry per lane and step
constexpr int kLayoutFlat = 1;  // the staged entries' products as one flat list
constexpr int kLayoutVec = 2;   // a group per B row, four consecutive entries per lane and step

// Four consecutive B entries [q, q + 4) with q a multiple of 4: values with
// one 16-byte load, column ids with one 4-, 8- or 16-byte load (1-, 2- or
// 4-byte ids); the arrays are 16-byte aligned (checked by the host). A chunk
// that would pass the end of B (bend = nnz(B)) is read entry by entry.
template <typename T, typename BR>
__device__ __forceinline__ void load_chunk4(const BR& br, int q, int bend, int (&j)[4], T (&v)[4]) {
  using IdxT = typename BR::Idx;
  if (q + 4 <= bend) {
    const int4 w4 = *reinterpret_cast<const int4*>((const T*)br.v + q);
    v[0] = __builtin_bit_cast(T, w4.x);
    v[1] = __builtin_bit_cast(T, w4.y);
    v[2] = __builtin_bit_cast(T, w4.z);
    v[3] = __builtin_bit_cast(T, w4.w);
    const IdxT* ids = br.ci + q;
    if constexpr (sizeof(IdxT) == 1) {
      const uint32_t w = *reinterpret_cast<const uint32_t*>(ids);
      j[0] = (int)(w & 0xffu);
      j[1] = (int)((w >> 8) & 0xffu);
      j[2] = (int)((w >> 16) & 0xffu);
      j[3] = (int)(w >> 24);
    } else if constexpr (sizeof(IdxT) == 2) {
      const uint2 w = *reinterpret_cast<const uint2*>(ids);
      j[0] = (int)(w.x & 0xffffu);
      j[1] = (int)(w.x >> 16);
      j[2] = (int)(w.y & 0xffffu);
      j[3] = (int)(w.y >> 16);
    } else {
      const int4 w = *reinterpret_cast<const int4*>(ids);
      j[0] = w.x;
      j[1] = w.y;
      j[2] = w.z;
      j[3] = w.w;
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      j[t] = 0;
      v[t] = T(0);
      if (q + t < bend) {
        j[t] = br.id(q + t);
        v[t] = br.template val<T>(q + t);
      }
    }
  }
}

// Add the entries of chunk [q, q + 4) that lie in the B row [q0, q1).
template <typename T>
__device__ __forceinline__ void add_chunk4(typename SemiringT<T>::acc* strip, int q, int q0, int q1, T a,
                                           const int (&j)[4], const T (&v)[4]) {
  using S = SemiringT<T>;
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (q + t >= q0 && q + t < q1) lds_add(&strip[j[t]], S::prod(a, v[t]));
}

// As accumulate_range_rows, but a lane of a group reads 4-entry chunks of
// the B row (chunk starts aligned to 4 entries: gl, gl + GL, ... counted from
// the chunk holding the row's first entry), so one load instruction covers
// four products and a wavefront keeps four times the B row bytes in flight.
template <int GL, typename T, typename BR>
__device__ __forceinline__ void accumulate_range_vec(const Problem& pr, int p_begin, int p_end, int wstart, int wstride,
                                                     typename SemiringT<T>::acc* strip, int4* stage) {
  constexpr int GPW = kWave / GL;
  constexpr int U = kHeavyUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  const int grp = lane / GL, gl = lane % GL;
  const T* __restrict__ aval = (const T*)pr.aval;
  const BR br(pr);
  const int bend = pr.brp[pr.n];

  for (int base = p_begin + kWave * wstart; base < p_end; base += kWave * wstride) {
    const int nb = min(kWave, p_end - base);
    int4 e = make_int4(0, 0, 0, 0);
    if (lane < nb) {
      const int2 bnd = entry_bounds(pr, base + lane);
      T a = aval[base + lane];
      e.x = bnd.x;
      e.y = bnd.y;
      e.z = __builtin_bit_cast(int32_t, a);
    }
    wave_sync();
    stage[lane] = e;
    wave_sync();
    for (int s = 0; s < nb; s += U * GPW) {
      int q[U], q0[U], q1[U];
      T av[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = s + u * GPW + grp;
        int4 r = make_int4(0, 0, 0, 0);
        if (src < nb) r = stage[src];
        q0[u] = r.x;
        q1[u] = r.y;
        q[u] = (r.x & ~3) + 4 * gl;
        av[u] = __builtin_bit_cast(T, r.z);
      }
      int jj[U][4];
      T bv[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] < q1[u]) load_chunk4<T>(br, q[u], bend, jj[u], bv[u]);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] < q1[u]) add_chunk4<T>(strip, q[u], q0[u], q1[u], av[u], jj[u], bv[u]);
#pragma unroll
      for (int u = 0; u < U; ++u)
        for (int qq = q[u] + 4 * GL; qq < q1[u]; qq += 4 * GL) {
          int j1[4];
          T v1[4];
          load_chunk4<T>(br, qq, bend, j1, v1);
          add_chunk4<T>(strip, qq, q0[u], q1[u], av[u], j1, v1);
        }
    }
    wave_sync();
  }
}

// Product layout of a wavefront's batch.
template <int GL, typename T, typename BR, int LAYOUT>
__device__ __forceinline__ void accumulate_range(const Problem& pr, int p_begin, int p_end, int wstart, int wstride,
                                                 typename SemiringT<T>::acc* strip, int4* stage) {
  if constexpr (LAYOUT == kLayoutFlat)
    accumulate_range_flat<T, BR>(pr, p_begin, p_end, wstart, wstride, strip, stage);
  else if constexpr (LAYOUT == kLayoutVec)
    accumulate_range_vec<GL, T, BR>(pr, p_begin, p_end, wstart, wstride, strip, stage);
  else
    accumulate_range_rows<GL, T, BR>(pr, p_begin, p_end, wstart, wstride, strip, stage);
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
template <int GL, typename T, typename BR>
__device__ __forceinline__ void accumulate_light_rows(const Problem& pr, int p0, int p1,
                                                 typename SemiringT<T>::acc* strip, int4* stage, int gl) {
  using S = SemiringT<T>;
  constexpr int U = kLightUnroll;
  const T* __restrict__ aval = (const T*)pr.aval;
  const BR br(pr);
  for (int base = p0; base < p1; base += GL) {
    const int nb = min(GL, p1 - base);
    int4 e = make_int4(0, 0, 0, 0);
    if (gl < nb) {
      const int2 bnd = entry_bounds(pr, base + gl);
      e.x = bnd.x;
      e.y = bnd.y;
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
          jj[u] = br.id(q[u]);
          bv[u] = br.template val<T>(q[u]);
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] < qe[u]) lds_add(&strip[jj[u]], S::prod(av[u], bv[u]));
#pragma unroll
      for (int u = 0; u < U; ++u)
        for (int qq = q[u] + GL; qq < qe[u]; qq += GL) lds_add(&strip[br.id(qq)], S::prod(av[u], br.template val<T>(qq)));
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
template <int GL, typename T, typename BR>
__device__ __forceinline__ void accumulate_light_flat(const Problem& pr, int p0, int p1,
                                                 typename SemiringT<T>::acc* strip, int4* stage, int gl) {
  using S = SemiringT<T>;
  constexpr int U = kLightUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  const T* __restrict__ aval = (const T*)pr.aval;
  const BR br(pr);
  for (int base = p0; base < p1; base += GL) {
    const int nb = min(GL, p1 - base);
    int q0 = 0, len = 0;
    T a = T(0);
    if (gl < nb) {
      const int2 bnd = entry_bounds(pr, base + gl);
      a = aval[base + gl];
      q0 = bnd.x;
      len = bnd.y - q0;
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
          jj[u] = br.id(q[u]);
          bv[u] = br.template val<T>(q[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] >= 0) lds_add(&strip[jj[u]], S::prod(av[u], bv[u]));
    }
    wave_sync();
  }
}

// As accumulate_light_rows, with 4-entry chunks of each B row per lane (see
// accumulate_range_vec).
template <int GL, typename T, typename BR>
__device__ __forceinline__ void accumulate_light_vec(const Problem& pr, int p0, int p1,
                                                     typename SemiringT<T>::acc* strip, int4* stage, int gl) {
  constexpr int U = kLightUnroll;
  const T* __restrict__ aval = (const T*)pr.aval;
  const BR br(pr);
  const int bend = pr.brp[pr.n];
  for (int base = p0; base < p1; base += GL) {
    const int nb = min(GL, p1 - base);
    int4 e = make_int4(0, 0, 0, 0);
    if (gl < nb) {
      const int2 bnd = entry_bounds(pr, base + gl);
      e.x = bnd.x;
      e.y = bnd.y;
      e.z = __builtin_bit_cast(int32_t, aval[base + gl]);
    }
    wave_sync();
    stage[gl] = e;
    wave_sync();
    for (int s = 0; s < nb; s += U) {
      int q[U], q0[U], q1[U];
      T av[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int4 r = make_int4(0, 0, 0, 0);
        if (s + u < nb) r = stage[s + u];
        q0[u] = r.x;
        q1[u] = r.y;
        q[u] = (r.x & ~3) + 4 * gl;
        av[u] = __builtin_bit_cast(T, r.z);
      }
      int jj[U][4];
      T bv[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] < q1[u]) load_chunk4<T>(br, q[u], bend, jj[u], bv[u]);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (q[u] < q1[u]) add_chunk4<T>(strip, q[u], q0[u], q1[u], av[u], jj[u], bv[u]);
#pragma unroll
      for (int u = 0; u < U; ++u)
        for (int qq = q[u] + 4 * GL; qq < q1[u]; qq += 4 * GL) {
          int j1[4];
          T v1[4];
          load_chunk4<T>(br, qq, bend, j1, v1);
          add_chunk4<T>(strip, qq, q0[u], q1[u], av[u], j1, v1);
        }
    }
    wave_sync();
  }
}

// Product layout of a lane group's row.
template <int GL, typename T, typename BR, int LAYOUT>
__device__ __forceinline__ void accumulate_light(const Problem& pr, int p0, int p1,
                                                 typename SemiringT<T>::acc* strip, int4* stage, int gl) {
  if constexpr (LAYOUT == kLayoutFlat)
    accumulate_light_flat<GL, T, BR>(pr, p0, p1, strip, stage, gl);
  else if constexpr (LAYOUT == kLayoutVec)
    accumulate_light_vec<GL, T, BR>(pr, p0, p1, strip, stage, gl);
  else
    accumulate_light_rows<GL, T, BR>(pr, p0, p1, strip, stage, gl);
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
