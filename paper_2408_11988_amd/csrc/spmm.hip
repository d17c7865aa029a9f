// Sparse A times dense tall-and-skinny B (SpMM), the alternative that
// Sec. V-C measures TS-SpGEMM against: C = A B with B and C dense n x d
// (row-major), plus-times over FP32 inputs with FP64 sums rounded once.
// Every A entry reads a whole B row of d values, zeros included, so it pays
// against TS-SpGEMM only when B is dense enough; bench.py measures where.
//
// A group of GL lanes owns one work item; lane gl owns the VEC-wide column
// chunks gl, gl + GL, ... (M chunks, FP64 sums in registers; VEC = 4, 2 or 1
// columns: the widest access B and C allow). The group stages GL of the item's A
// entries at once (coalesced) and reads one B row per step, as one VEC-wide
// load per chunk. A row of at most kSpmmChunk A entries is one item
// and written directly; a longer row is cut into items of kSpmmChunk entries
// whose FP64 partial rows a second kernel adds in chunk order. Every group
// takes exactly one item and the items are launched as one grid (chunks of
// long rows first), so the hardware's workgroup dispatch balances the skewed
// row lengths of power-law inputs. All summation orders are fixed.
#include <mutex>
#include <string>

#include "api_internal.hpp"
#include "dev_numeric.hpp"

namespace tss {

constexpr int kSpmmChunk = 128;  // A entries per work item of a long row
struct SpmmParams {
  int64_t n, d, ldb, ldc;
  const int32_t* arp;
  const int32_t* aci;
  const float* aval;
  const float* B;
  float* C;
  int2* chunks;        // (row, chunk index) of each chunk slot
  int4* long_rows;     // (row, first slot, chunk count, -) of each long row
  double* partial;     // chunk slot x d
  int32_t* counters;   // [0] chunk slots used, [1] long rows
  int64_t slot_items;  // groups reserved for chunk slots (a bound on their count)
};

// Long rows: reserve one slot per chunk. Each wavefront sums its rows' chunk
// counts with a shuffle scan and reserves slots and long-row records for all
// of them with one 64-bit atomic (chunks in the low word, rows in the high
// word). The order of reservations does not matter: a row's slots are
// consecutive and added in chunk order.
__global__ void k_spmm_classify(SpmmParams sp) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x - lane); i0 < sp.n; i0 += stride) {
    const int64_t i = i0 + lane;
    int nc = 0;
    if (i < sp.n) {
      const int len = sp.arp[i + 1] - sp.arp[i];
      if (len > kSpmmChunk) nc = (len + kSpmmChunk - 1) / kSpmmChunk;
    }
    const uint64_t longs = __ballot(nc > 0);
    if (longs == 0) continue;
    int incl = nc;  // inclusive scan of the chunk counts over the wavefront
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const int t = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += t;
    }
    const int total = __shfl(incl, kWave - 1, kWave);
    unsigned long long base = 0;
    if (lane == 0)
      base = atomicAdd(reinterpret_cast<unsigned long long*>(sp.counters),
                       ((unsigned long long)__popcll(longs) << 32) | (unsigned)total);
    const int first0 = __shfl((int)(unsigned)base, 0, kWave);
    const int row0 = __shfl((int)(unsigned)(base >> 32), 0, kWave);
    if (nc > 0) {
      const int first = first0 + incl - nc;
      sp.long_rows[row0 + lanes_below(longs)] = make_int4((int)i, first, nc, 0);
      for (int c = 0; c < nc; ++c) sp.chunks[first + c] = make_int2((int)i, c);
    }
  }
}

template <int VEC>
struct VecF;
template <>
struct VecF<4> {
  using type = float4;
};
template <>
struct VecF<2> {
  using type = float2;
};
template <>
struct VecF<1> {
  using type = float;
};

template <int VEC>
__device__ __forceinline__ void fma_vec(double* acc, float a, const typename VecF<VEC>::type& b) {
  if constexpr (VEC == 4) {
    acc[0] += (double)a * (double)b.x;
    acc[1] += (double)a * (double)b.y;
    acc[2] += (double)a * (double)b.z;
    acc[3] += (double)a * (double)b.w;
  } else if constexpr (VEC == 2) {
    acc[0] += (double)a * (double)b.x;
    acc[1] += (double)a * (double)b.y;
  } else {
    acc[0] += (double)a * (double)b;
  }
}

// Sums of A entries [p0, p1) of one row times B rows into acc (M chunks of
// VEC columns, lane gl of a GL-lane group). Entries are staged GL at a time
// and broadcast inside the group with shuffles; each step reads one B row.
// (Several B rows in flight per group measured slower: 0.92 ms for eight
// against 0.63 ms for one at R-MAT 18 x 128, where more groups share each
// wavefront instead.)
template <int GL, int VEC, int M>
__device__ __forceinline__ void spmm_range(const SpmmParams& sp, int p0, int p1, int gl, double (&acc)[M][VEC]) {
  using V = typename VecF<VEC>::type;
  const int lane = threadIdx.x & (kWave - 1);
  const int g0 = lane & ~(GL - 1);
  for (int base = p0; base < p1; base += GL) {
    const int nb = min(GL, p1 - base);
    int kk = 0;
    float av = 0.0f;
    if (gl < nb) {
      kk = sp.aci[base + gl];
      av = sp.aval[base + gl];
    }
    for (int e = 0; e < nb; ++e) {
      const int k = __shfl(kk, g0 + e, kWave);
      const float a = __shfl(av, g0 + e, kWave);
      const V* row = reinterpret_cast<const V*>(sp.B + (int64_t)k * sp.ldb);
#pragma unroll
      for (int m = 0; m < M; ++m)
        if ((int64_t)(m * GL + gl) * VEC < sp.d) fma_vec<VEC>(acc[m], a, row[m * GL + gl]);
    }
  }
}

// One item per group: chunk slots s < slot_items (those beyond the used
// count exit), then rows i = item - slot_items (long rows exit: their
// chunks cover them).
template <int GL, int VEC, int M>
__global__ __launch_bounds__(kBlock) void k_spmm_items(SpmmParams sp) {
  constexpr int G = kBlock / GL;
  const int grp = threadIdx.x / GL, gl = threadIdx.x % GL;
  const int64_t item = (int64_t)blockIdx.x * G + grp;
  double acc[M][VEC];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[m][v] = 0.0;
  if (item < sp.slot_items) {
    if (item >= sp.counters[0]) return;
    const int2 ch = sp.chunks[item];
    const int a0 = sp.arp[ch.x], a1 = sp.arp[ch.x + 1];
    const int p0 = a0 + ch.y * kSpmmChunk;
    const int p1 = min(a1, p0 + kSpmmChunk);
    spmm_range<GL, VEC, M>(sp, p0, p1, gl, acc);
    double* dst = sp.partial + item * sp.d;
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int64_t c = (int64_t)(m * GL + gl) * VEC + v;
        if (c < sp.d) dst[c] = acc[m][v];
      }
    return;
  }
  const int64_t i = item - sp.slot_items;
  if (i >= sp.n) return;
  const int p0 = sp.arp[i], p1 = sp.arp[i + 1];
  if (p1 - p0 > kSpmmChunk) return;
  spmm_range<GL, VEC, M>(sp, p0, p1, gl, acc);
  float* crow = sp.C + i * sp.ldc;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int64_t c = (int64_t)(m * GL + gl) * VEC;
    if (c < sp.d) {
      if constexpr (VEC == 4)
        reinterpret_cast<float4*>(crow)[m * GL + gl] =
            make_float4((float)acc[m][0], (float)acc[m][1], (float)acc[m][2], (float)acc[m][3]);
      else if constexpr (VEC == 2)
        reinterpret_cast<float2*>(crow)[m * GL + gl] = make_float2((float)acc[m][0], (float)acc[m][1]);
      else
        crow[c] = (float)acc[m][0];
    }
  }
}

// Long rows: add the chunk partials in chunk order and write the row (the
// loads of eight chunks are issued before their sums).
__global__ void k_spmm_finalize(SpmmParams sp) {
  const int nrows = sp.counters[1];
  for (int r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int4 lr = sp.long_rows[r];
    const double* part = sp.partial + (int64_t)lr.y * sp.d;
    for (int64_t c = threadIdx.x; c < sp.d; c += blockDim.x) {
      double s = 0.0;
      int q = 0;
      for (; q + 8 <= lr.z; q += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(q + u) * sp.d + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
      }
      for (; q < lr.z; ++q) s += part[(int64_t)q * sp.d + c];
      sp.C[(int64_t)lr.x * sp.ldc + c] = (float)s;
    }
  }
}

template <int GL, int VEC, int M>
static void launch_spmm_t(const SpmmParams& sp, hipStream_t st) {
  constexpr int G = kBlock / GL;
  const int64_t g = (sp.slot_items + sp.n + G - 1) / G;
  k_spmm_items<GL, VEC, M><<<(unsigned)g, kBlock, 0, st>>>(sp);
  k_spmm_finalize<<<1024, 256, 0, st>>>(sp);
}

template <int VEC>
static int launch_spmm_v(const SpmmParams& sp, hipStream_t st) {
  const int64_t chunks = (sp.d + VEC - 1) / VEC;  // VEC-wide column chunks
  if (chunks <= 8)
    launch_spmm_t<8, VEC, 1>(sp, st);
  else if (chunks <= 16)
    launch_spmm_t<16, VEC, 1>(sp, st);
  else if (chunks <= 32)
    launch_spmm_t<32, VEC, 1>(sp, st);
  else if (chunks <= 64)
    launch_spmm_t<64, VEC, 1>(sp, st);
  else if (chunks <= 128)
    launch_spmm_t<64, VEC, 2>(sp, st);
  else if (chunks <= 256)
    launch_spmm_t<64, VEC, 4>(sp, st);
  else if (chunks <= 512)
    launch_spmm_t<64, VEC, 8>(sp, st);
  else if (chunks <= 1024)
    launch_spmm_t<64, VEC, 16>(sp, st);
  else {
    set_error("spmm: d too large");
    return TSSPGEMM_ERR_UNSUPPORTED;
  }
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// Argument checks shared by both entry points; *nothing is set when there is
// no work (n = 0 or d = 0).
static int check_spmm(const tsspgemm_csr* A, const float* B, int64_t d, int64_t ldb, const float* C, int64_t ldc) {
  int rc;
  if ((rc = check_csr(A, "A", true))) return rc;
  if (A->nrows != A->ncols) {
    set_error("A must be square (n x n)");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (d < 0 || ldb < d || ldc < d || (A->nrows > 0 && d > 0 && (!B || !C))) {
    set_error("spmm: bad d, leading dimensions or NULL B / C");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (d > kMaxDenseD) {
    set_error("spmm: d > 1024");
    return TSSPGEMM_ERR_UNSUPPORTED;
  }
  return TSSPGEMM_OK;
}

// Bounds on the chunk slots and long rows of A: a row of len > kSpmmChunk
// entries has ceil(len / kSpmmChunk) <= 2 len / kSpmmChunk chunks.
static int64_t spmm_chunk_cap(int64_t nnz) { return 2 * nnz / kSpmmChunk + 1; }
static int64_t spmm_long_cap(int64_t nnz) { return nnz / kSpmmChunk + 1; }

// Queues the classification, the item kernel and the finalize on `st`, with
// the workspace pointers already set in sp (counters zeroed here by a fill
// kernel, no memset node).
static int enqueue_spmm(SpmmParams& sp, hipStream_t st) {
  int rc;
  if ((rc = launch_zero_bytes(sp.counters, 16, st))) return rc;
  k_spmm_classify<<<grid_for(sp.n, 256) > 4096 ? 4096 : grid_for(sp.n, 256), 256, 0, st>>>(sp);
  TSS_CHECK_LAUNCH();
  // widest lane access that B and C allow: 16 bytes (fewer lanes per row, so
  // more rows per wavefront), else 8, else 4
  const auto fits = [&](int v) {
    return sp.d % v == 0 && sp.ldb % v == 0 && sp.ldc % v == 0 && ((uintptr_t)sp.B % (4 * v)) == 0 &&
           ((uintptr_t)sp.C % (4 * v)) == 0;
  };
  if (fits(4)) return launch_spmm_v<4>(sp, st);
  return fits(2) ? launch_spmm_v<2>(sp, st) : launch_spmm_v<1>(sp, st);
}

static SpmmParams spmm_params(const tsspgemm_csr* A, const float* B, int64_t d, int64_t ldb, float* C, int64_t ldc) {
  SpmmParams sp{};
  sp.n = A->nrows;
  sp.d = d;
  sp.ldb = ldb;
  sp.ldc = ldc;
  sp.arp = A->rowptr;
  sp.aci = A->colidx;
  sp.aval = (const float*)A->vals;
  sp.B = B;
  sp.C = C;
  sp.slot_items = spmm_chunk_cap(A->nnz);
  return sp;
}

static int run_spmm(const tsspgemm_csr* A, const float* B, int64_t d, int64_t ldb, float* C, int64_t ldc,
                    hipStream_t st) {
  int rc;
  if ((rc = check_spmm(A, B, d, ldb, C, ldc))) return rc;
  const int64_t n = A->nrows, nnz = A->nnz;
  if (n == 0 || d == 0) return TSSPGEMM_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  Plan* p = cached_plan(dev);
  if (!p) {
    set_error("no workspace cache for this device");
    return TSSPGEMM_ERR_NOMEM;
  }
  std::lock_guard<std::mutex> lk(p->mu);
  StreamOrder so(p, st);
  if (so.rc) return so.rc;
  const int64_t chunk_cap = spmm_chunk_cap(nnz), long_cap = spmm_long_cap(nnz);
  if ((rc = p->sp_chunks.ensure((size_t)chunk_cap * sizeof(int2))) ||
      (rc = p->sp_rows.ensure((size_t)long_cap * sizeof(int4))) ||
      (rc = p->sp_partial.ensure((size_t)chunk_cap * d * 8)) || (rc = p->sp_ctr.ensure(16)))
    return rc;
  SpmmParams sp = spmm_params(A, B, d, ldb, C, ldc);
  sp.chunks = (int2*)p->sp_chunks.p;
  sp.long_rows = (int4*)p->sp_rows.p;
  sp.partial = (double*)p->sp_partial.p;
  sp.counters = (int32_t*)p->sp_ctr.p;
  return enqueue_spmm(sp, st);
}

// ---------------------------------------------------------------- allocation-free variant

// The workspace of tsspgemm_spmm_noalloc: counters, chunk list, long-row
// records and FP64 partial rows, carved from one fixed device array. Each
// GPU holds its own copy (allocated with the code object, kept until the
// process ends); the host reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kSpmmScratchBytes = (size_t)TSSPGEMM_SPMM_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kSpmmScratchBytes];

constexpr int kScratchMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchMaxDevices];  // device address of `scratch` on each device, once looked up

// Device address of this device's scratch array (looked up once per device,
// with that device current).
static int scratch_address(void** out) {
  int dev = 0;
  TSS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchMaxDevices) {
    set_error("spmm_noalloc: device ordinal beyond the supported 64");
    return TSSPGEMM_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return TSSPGEMM_ERR_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TSSPGEMM_OK;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Bytes of scratch an n x n A with nnz entries needs at width d.
static size_t spmm_scratch_bytes(int64_t nnz, int64_t d) {
  const int64_t chunk_cap = spmm_chunk_cap(nnz), long_cap = spmm_long_cap(nnz);
  return 256 + align256((size_t)chunk_cap * sizeof(int2)) + align256((size_t)long_cap * sizeof(int4)) +
         align256((size_t)chunk_cap * d * 8);
}

static int run_spmm_noalloc(const tsspgemm_csr* A, const float* B, int64_t d, int64_t ldb, float* C, int64_t ldc,
                            hipStream_t st) {
  int rc;
  if ((rc = check_spmm(A, B, d, ldb, C, ldc))) return rc;
  const int64_t n = A->nrows, nnz = A->nnz;
  if (n == 0 || d == 0) return TSSPGEMM_OK;
  const size_t need = spmm_scratch_bytes(nnz, d);
  if (need > kSpmmScratchBytes) {
    set_error("spmm_noalloc: this A and d need " + std::to_string(need) + " bytes of scratch; the maximum is " +
              std::to_string(kSpmmScratchBytes) + " (about nnz(A) * d / 8 bytes); use tsspgemm_spmm");
    return TSSPGEMM_ERR_CAPACITY;
  }
  void* base = nullptr;
  if ((rc = scratch_address(&base))) return rc;
  char* p = (char*)base;
  const int64_t chunk_cap = spmm_chunk_cap(nnz), long_cap = spmm_long_cap(nnz);
  SpmmParams sp = spmm_params(A, B, d, ldb, C, ldc);
  sp.counters = (int32_t*)p;
  p += 256;
  sp.chunks = (int2*)p;
  p += align256((size_t)chunk_cap * sizeof(int2));
  sp.long_rows = (int4*)p;
  p += align256((size_t)long_cap * sizeof(int4));
  sp.partial = (double*)p;
  return enqueue_spmm(sp, st);
}

}  // namespace tss

extern "C" int tsspgemm_spmm(const tsspgemm_csr* A, const float* B, int64_t d, int64_t ldb, float* C, int64_t ldc,
                             void* stream) {
  try {
    return tss::run_spmm(A, B, d, ldb, C, ldc, (hipStream_t)stream);
  } catch (...) {
    tss::set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}

extern "C" int tsspgemm_spmm_noalloc(const tsspgemm_csr* A, const float* B, int64_t d, int64_t ldb, float* C,
                                     int64_t ldc, void* stream) {
  try {
    return tss::run_spmm_noalloc(A, B, d, ldb, C, ldc, (hipStream_t)stream);
  } catch (...) {
    tss::set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}
