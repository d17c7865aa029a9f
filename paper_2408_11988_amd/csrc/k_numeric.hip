// Numeric phase of row-wise Gustavson TS-SpGEMM (Sec. III-A, Eq. 1):
// C(i,:) = sum over k in pat(A_i) of A(i,k) B(k,:), with the dense accumulator
// (SPA) of width d that Sec. III-C prefers for d <= 1024. On gfx950 a strip of
// d accumulators lives in LDS (FP64 for the FP32 semiring: every FP32 x FP32
// product is exact in FP64 and is added with the native ds_add_f64, then
// rounded once to FP32 at the end).
//
// The kernel is bound by the latency of dependent gathers (A entry -> B row
// pointers -> B row), so the work layout is about keeping many rows in flight.
// Rows are binned by their product count flops_i (Sec. II-A):
//  * light rows: a group of GL lanes owns one row and one strip, so 256/GL
//    rows per workgroup are in flight; groups walk the binned list with a
//    grid stride, so neighbouring groups get rows of similar cost;
//  * wavefront rows: one wavefront per row, four rows per workgroup;
//  * workgroup rows: the four wavefronts of a workgroup share the row, each
//    accumulating a private strip, summed in a fixed order;
//  * split rows: chunks of A entries go to separate workgroups, each writes
//    its partial strip to global memory; a second kernel adds the partials in
//    chunk order and writes the row.
// Every order of addition is fixed, so results are reproducible run to run.
// Streaming B: a group of GL lanes reads one B row (GL consecutive entries per
// step, coalesced); several A entries are unrolled so that several B rows are
// in flight per group.
// Output: the row's pattern is already known as a bitmap (symbolic phase);
// a lane owns column j of a chunk, and its output slot is the popcount of the
// set bits below it, so columns come out sorted without a sort.
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

// Accumulate entries [p_begin, p_end) of one A row into `strip`, taking
// 64-entry batches number wstart, wstart + wstride, ... (one wavefront).
template <int GL, typename T>
__device__ __forceinline__ void accumulate_range(const Problem& pr, int p_begin, int p_end, int wstart, int wstride,
                                                 typename SemiringT<T>::acc* strip, int4* stage) {
  using S = SemiringT<T>;
  constexpr int GPW = kWave / GL;
  constexpr int U = kHeavyUnroll;
  const int lane = threadIdx.x & (kWave - 1);
  const int grp = lane / GL, gl = lane % GL;
  const int32_t* __restrict__ aci = pr.aci;
  const T* __restrict__ aval = (const T*)pr.aval;
  const int32_t* __restrict__ brp = pr.brp;
  const int32_t* __restrict__ bci = pr.bci;
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
      int q[U], qe[U], jj[U];
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

template <int GL, typename T>
__global__ __launch_bounds__(kBlock) void k_numeric(NumParams np) {
  using S = SemiringT<T>;
  using Acc = typename S::acc;
  extern __shared__ __align__(16) unsigned char smem[];
  const Problem& pr = np.pr;
  const int d = pr.d;
  Acc* strips = (Acc*)smem;
  int4* stage = (int4*)(smem + (size_t)kWavesPerBlock * d * sizeof(Acc));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int g = blockIdx.x;
  const bool wg_mode = g < np.n_wg_items;
  Item it{-1, 0, 0, 0};
  bool valid;
  if (wg_mode) {
    it = np.items[g];
    valid = true;
  } else {
    const int64_t idx = (int64_t)np.n_wg_items + 4 * (int64_t)(g - np.n_wg_items) + wave;
    valid = idx < np.n_heavy_records;
    if (valid) it = np.items[idx];
  }
  Acc* strip = strips + wave * d;
  for (int j = lane; j < d; j += kWave) strip[j] = Acc(0);
  __syncthreads();
  if (valid) {
    if (wg_mode)
      accumulate_range<GL, T>(pr, it.p0, it.p1, wave, kWavesPerBlock, strip, stage + wave * kWave);
    else
      accumulate_range<GL, T>(pr, it.p0, it.p1, 0, 1, strip, stage + wave * kWave);
  }
  __syncthreads();
  if (wg_mode) {
    for (int j = threadIdx.x; j < d; j += kBlock)
      strips[j] = S::add(S::add(S::add(strips[j], strips[d + j]), strips[2 * d + j]), strips[3 * d + j]);
    __syncthreads();
    if (it.aux != kNoSlot) {
      // split chunk: partial sums to its slot (added up by k_split_finalize)
      if constexpr (sizeof(Acc) == 8) {
        double* dst = np.partial + (int64_t)it.aux * d;
        for (int j = threadIdx.x; j < d; j += kBlock) dst[j] = strips[j];
      } else {
        int32_t* dst = np.ipartial + (int64_t)it.aux * d;
        for (int j = threadIdx.x; j < d; j += kBlock) dst[j] = strips[j];
      }
    } else {
      emit_row<T>(pr, it.row, strips, wave, kWavesPerBlock);
    }
  } else if (valid) {
    emit_row<T>(pr, it.row, strip, 0, 1);
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

template <int GL, typename T>
__global__ __launch_bounds__(kBlock) void k_numeric_light(NumParams np) {
  using S = SemiringT<T>;
  using Acc = typename S::acc;
  constexpr int G = kBlock / GL;  // rows in flight per workgroup
  constexpr int U = kLightUnroll;
  extern __shared__ __align__(16) unsigned char smem[];
  const Problem& pr = np.pr;
  const int d = pr.d;
  const int grp = threadIdx.x / GL, gl = threadIdx.x % GL;
  Acc* strip = (Acc*)smem + grp * d;
  const int32_t* __restrict__ aci = pr.aci;
  const T* __restrict__ aval = (const T*)pr.aval;
  const int32_t* __restrict__ brp = pr.brp;
  const int32_t* __restrict__ bci = pr.bci;
  const T* __restrict__ bval = (const T*)pr.bval;
  const Item* items = np.items + np.n_heavy_records;
  const int64_t stride = (int64_t)gridDim.x * G;
  for (int64_t t = (int64_t)blockIdx.x * G + grp; t < np.n_light; t += stride) {
    const Item it = items[t];
    for (int j = gl; j < d; j += GL) strip[j] = Acc(0);
    wave_sync();
    for (int p = it.p0; p < it.p1; p += U) {
      int k[U], q[U], qe[U], jj[U];
      T av[U], bv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool v = p + u < it.p1;
        k[u] = v ? aci[p + u] : -1;
        av[u] = v ? aval[p + u] : T(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        q[u] = 0;
        qe[u] = 0;
        if (k[u] >= 0) {
          q[u] = brp[k[u]] + gl;
          qe[u] = brp[k[u] + 1];
        }
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
    emit_group<GL, T>(pr, it.row, strip, gl);
    wave_sync();
  }
}

// ---------------------------------------------------------------- launch

static size_t acc_bytes(int sr) { return sr == TSSPGEMM_PLUS_TIMES_F32 ? 8 : 4; }

int light_group_lanes(int group_lanes, int64_t d, int sr) {
  // strips of all groups of a workgroup must fit 64 KB of LDS
  int gl = group_lanes;
  while (gl < 64 && (size_t)(kBlock / gl) * d * acc_bytes(sr) > 65536) gl <<= 1;
  return gl;
}

static int64_t light_grid(int64_t n_light, int gl) {
  const int64_t per_block = kBlock / gl;
  int64_t g = (n_light + per_block - 1) / per_block;
  const int64_t cap = 256 * 8;  // CUs x resident workgroups
  return g < cap ? g : cap;
}

int launch_numeric(int sr, int group_lanes, const NumParams& np, int64_t n_grid, hipStream_t st) {
  const size_t ab = acc_bytes(sr);
  if (n_grid > 0) {
    const size_t lds = (size_t)kWavesPerBlock * np.pr.d * ab + kWavesPerBlock * kWave * sizeof(int4);
#define TSS_NUM_CASE(GLV)                                                 \
  case GLV:                                                               \
    if (sr == TSSPGEMM_PLUS_TIMES_F32)                                    \
      k_numeric<GLV, float><<<(unsigned)n_grid, kBlock, lds, st>>>(np);   \
    else                                                                  \
      k_numeric<GLV, int32_t><<<(unsigned)n_grid, kBlock, lds, st>>>(np); \
    break;
    switch (group_lanes) {
      TSS_NUM_CASE(4)
      TSS_NUM_CASE(8)
      TSS_NUM_CASE(16)
      TSS_NUM_CASE(32)
      TSS_NUM_CASE(64)
      default:
        set_error("numeric: group_lanes must be 4, 8, 16, 32 or 64");
        return TSSPGEMM_ERR_INVALID_ARG;
    }
#undef TSS_NUM_CASE
    TSS_CHECK_LAUNCH();
  }
  if (np.n_light > 0) {
    const int gl = light_group_lanes(group_lanes, np.pr.d, sr);
    const unsigned g = (unsigned)light_grid(np.n_light, gl);
    const size_t lds = (size_t)(kBlock / gl) * np.pr.d * ab;
#define TSS_LIGHT_CASE(GLV)                                      \
  case GLV:                                                      \
    if (sr == TSSPGEMM_PLUS_TIMES_F32)                           \
      k_numeric_light<GLV, float><<<g, kBlock, lds, st>>>(np);   \
    else                                                         \
      k_numeric_light<GLV, int32_t><<<g, kBlock, lds, st>>>(np); \
    break;
    switch (gl) {
      TSS_LIGHT_CASE(4)
      TSS_LIGHT_CASE(8)
      TSS_LIGHT_CASE(16)
      TSS_LIGHT_CASE(32)
      TSS_LIGHT_CASE(64)
      default:
        set_error("numeric: bad light group width");
        return TSSPGEMM_ERR_INVALID_ARG;
    }
#undef TSS_LIGHT_CASE
    TSS_CHECK_LAUNCH();
  }
  return TSSPGEMM_OK;
}

// Split rows: add the chunks' partial strips in chunk order, then emit.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_split_finalize(Problem pr, const SplitRow* rows, const double* partial,
                                                           const int32_t* ipartial) {
  using S = SemiringT<T>;
  using Acc = typename S::acc;
  extern __shared__ __align__(16) unsigned char smem[];
  Acc* strip = (Acc*)smem;
  const SplitRow r = rows[blockIdx.x];
  const int d = pr.d;
  for (int j = threadIdx.x; j < d; j += kBlock) {
    Acc s = Acc(0);
    for (int c = 0; c < r.count; ++c) {
      if constexpr (sizeof(Acc) == 8)
        s = S::add(s, partial[(int64_t)(r.first + c) * d + j]);
      else
        s = S::add(s, ipartial[(int64_t)(r.first + c) * d + j]);
    }
    strip[j] = s;
  }
  __syncthreads();
  emit_row<T>(pr, r.row, strip, threadIdx.x >> 6, kWavesPerBlock);
}

int launch_split_finalize(int sr, const Problem& pr, const SplitRow* rows, int32_t nrows, const double* partial,
                          const int32_t* ipartial, hipStream_t st) {
  if (nrows == 0) return TSSPGEMM_OK;
  if (sr == TSSPGEMM_PLUS_TIMES_F32)
    k_split_finalize<float><<<nrows, kBlock, (size_t)pr.d * 8, st>>>(pr, rows, partial, ipartial);
  else
    k_split_finalize<int32_t><<<nrows, kBlock, (size_t)pr.d * 4, st>>>(pr, rows, partial, ipartial);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// (AND, OR): the output is the pattern alone. Lane = (row, word): each lane
// writes the set bits of one bitmap word, at the row start plus the popcount
// of the row's earlier words (segmented scan over the row's wp lanes).
__global__ void k_emit_pattern(Problem pr) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int wp = pr.wp;
  const int64_t row = t / wp;
  const int w = (int)(t % wp);
  const bool ok = row < pr.n;
  uint32_t word = ok ? pr.cbits[row * wp + w] : 0u;
  const int c = __popc(word);
  int x = c;
  const int lane = threadIdx.x & 63;
  for (int o = 1; o < wp; o <<= 1) {
    const int y = __shfl_up(x, o, kWave);
    if ((lane % wp) >= o) x += y;
  }
  if (!ok || word == 0u) return;
  int pos = pr.crp[row] + x - c;
  while (word) {
    const int b = __ffs(word) - 1;
    pr.cci[pos++] = 32 * w + b;
    word &= word - 1;
  }
}

int launch_emit_pattern(const Problem& pr, hipStream_t st) {
  const int64_t lanes = (int64_t)pr.n * pr.wp;
  if (lanes == 0) return TSSPGEMM_OK;
  k_emit_pattern<<<grid_for(lanes, 256), 256, 0, st>>>(pr);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// ================================================================ binning (numeric)

// Work class by product count: 3 = light (a lane group), 2 = one wavefront,
// 1 = one workgroup, 0 = split into chunks of at least kMinChunk A entries.
constexpr int kMinChunk = 64;

__device__ __forceinline__ int num_class(int64_t f, const NumThresholds& th) {
  return f <= th.light_max ? 3 : (f <= th.wave_max ? 2 : (f <= th.split ? 1 : 0));
}
__device__ __forceinline__ int num_bin(int64_t work) {
  const int e = 63 - __clzll((unsigned long long)work);
  const int b = kBins - 1 - e;
  return b < 0 ? 0 : b;
}
__device__ __forceinline__ int chunk_entries(int m, int64_t f, int64_t split) {
  const int64_t want = (f + split - 1) / split;  // chunks by products
  int ce = (int)((m + want - 1) / want);
  return ce < kMinChunk ? kMinChunk : ce;
}

__global__ void k_num_bin_count(Problem pr, NumThresholds th, Counters* ctr) {
  __shared__ int32_t hist[kNumClasses * kBins];
  for (int t = threadIdx.x; t < kNumClasses * kBins; t += blockDim.x) hist[t] = 0;
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < pr.n) {
    const int64_t f = pr.flops[i];
    if (f > 0) {
      const int cls = num_class(f, th);
      if (cls == 0) {
        const int m = pr.arp[i + 1] - pr.arp[i];
        const int ce = chunk_entries(m, f, th.split);
        atomicAdd(&hist[0], (m + ce - 1) / ce);
      } else {
        atomicAdd(&hist[cls * kBins + num_bin(f)], 1);
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kNumClasses * kBins; t += blockDim.x)
    if (hist[t]) atomicAdd(&(&ctr->num_count[0][0])[t], hist[t]);
}

__global__ void k_num_bin_scan(Counters* ctr) {
  int32_t off = 0;
  int32_t tot[kNumClasses] = {0, 0, 0, 0};
  for (int c = 0; c < kNumClasses; ++c)
    for (int b = 0; b < kBins; ++b) {
      ctr->num_cursor[c][b] = off;
      off += ctr->num_count[c][b];
      tot[c] += ctr->num_count[c][b];
    }
  ctr->num_split_items = tot[0];
  ctr->num_block_items = tot[1];
  ctr->num_wave_rows = tot[2];
  ctr->num_light_rows = tot[3];
}

// Items are placed with one global reservation per (class, bin) per
// workgroup; the slot inside the workgroup's range comes from an LDS counter.
__global__ void k_num_bin_fill(Problem pr, NumThresholds th, Item* items, SplitRow* split_rows, Counters* ctr) {
  __shared__ int32_t cnt[kNumClasses * kBins], base[kNumClasses * kBins];
  __shared__ int32_t nsplit, split_base;
  for (int t = threadIdx.x; t < kNumClasses * kBins; t += blockDim.x) cnt[t] = 0;
  if (threadIdx.x == 0) nsplit = 0;
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int a = 0, m = 0, cls = 0, key = 0, count = 0, local = 0, ce = 0, slocal = 0;
  if (i < pr.n) {
    const int64_t f = pr.flops[i];
    if (f > 0) {
      a = pr.arp[i];
      m = pr.arp[i + 1] - a;
      cls = num_class(f, th);
      if (cls == 0) {
        ce = chunk_entries(m, f, th.split);
        count = (m + ce - 1) / ce;
        key = 0;
        slocal = atomicAdd(&nsplit, 1);
      } else {
        count = 1;
        key = cls * kBins + num_bin(f);
      }
      local = atomicAdd(&cnt[key], count);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kNumClasses * kBins; t += blockDim.x)
    if (cnt[t]) base[t] = atomicAdd(&(&ctr->num_cursor[0][0])[t], cnt[t]);
  if (threadIdx.x == 0 && nsplit) split_base = atomicAdd(&ctr->num_split_rows, nsplit);
  __syncthreads();
  if (count == 0) return;
  const int pos = base[key] + local;
  if (cls == 0) {
    for (int c = 0; c < count; ++c) {
      const int p0 = a + c * ce;
      items[pos + c] = Item{(int32_t)i, p0, min(a + m, p0 + ce), pos + c};
    }
    split_rows[split_base + slocal] = SplitRow{(int32_t)i, pos, count, 0};
  } else {
    items[pos] = Item{(int32_t)i, a, a + m, cls == 1 ? kNoSlot : 0};
  }
}

int launch_num_bin(const Problem& pr, const NumThresholds& th, Item* items, SplitRow* split_rows, Counters* ctr,
                   hipStream_t st) {
  if (pr.n > 0) {
    const unsigned g = grid_for(pr.n, 256);
    k_num_bin_count<<<g, 256, 0, st>>>(pr, th, ctr);
    k_num_bin_scan<<<1, 1, 0, st>>>(ctr);
    k_num_bin_fill<<<g, 256, 0, st>>>(pr, th, items, split_rows, ctr);
  } else {
    k_num_bin_scan<<<1, 1, 0, st>>>(ctr);
  }
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

}  // namespace tss
