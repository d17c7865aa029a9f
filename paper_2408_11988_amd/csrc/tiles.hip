// Column tiles of A and the merge of partial outputs (Sec. III-B, III-C,
// Algorithm 2). A tile here is a range of A's columns taken over every row
// (the tile height is the whole local row block on one GPU): the product of
// the tile with B only reads B's rows in that range. The partial products of
// the tiles are then merged row by row; the paper merges with a dense
// accumulator (SPA) when d is small, and so does this merge: a d-wide FP64
// strip and a d-bit pattern per row in LDS, the parts added in order, each
// output value rounded once.
#include "api_internal.hpp"
#include "dev_numeric.hpp"

namespace tss {

constexpr int kMergeMaxParts = 64;
constexpr int kTileWaves = 4;

struct MergeParts {
  int32_t count;
  int64_t n, d;
  const int32_t* rp[kMergeMaxParts];
  const int32_t* ci[kMergeMaxParts];
  const float* val[kMergeMaxParts];
};

// first position in [lo, hi) of aci whose column is >= c (aci sorted)
__device__ __forceinline__ int lower_col(const int32_t* __restrict__ aci, int lo, int hi, int32_t c) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (aci[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ void k_slice_count(int64_t n, const int32_t* __restrict__ arp, const int32_t* __restrict__ aci, int32_t c0,
                              int32_t c1, int32_t* __restrict__ cnt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int lo = lower_col(aci, arp[i], arp[i + 1], c0);
    const int hi = lower_col(aci, lo, arp[i + 1], c1);
    cnt[i] = hi - lo;
  }
}

// one wavefront per row: the row's entries in [c0, c1) copied to out_rp[i]
__global__ __launch_bounds__(kTileWaves * kWave) void k_slice_fill(int64_t n, const int32_t* __restrict__ arp,
                                                                   const int32_t* __restrict__ aci,
                                                                   const float* __restrict__ aval, int32_t c0,
                                                                   int32_t c1, const int32_t* __restrict__ out_rp,
                                                                   int32_t* __restrict__ out_ci,
                                                                   float* __restrict__ out_val) {
  const int lane = threadIdx.x % kWave;
  for (int64_t i = (int64_t)blockIdx.x * kTileWaves + threadIdx.x / kWave; i < n;
       i += (int64_t)gridDim.x * kTileWaves) {
    const int lo = lower_col(aci, arp[i], arp[i + 1], c0);
    const int len = out_rp[i + 1] - out_rp[i];
    const int64_t o = out_rp[i];
    for (int t = lane; t < len; t += kWave) {
      out_ci[o + t] = aci[lo + t];
      if (out_val) out_val[o + t] = aval[lo + t];
    }
  }
}

// Union pattern size of each row over the parts (d-bit pattern in LDS).
__global__ __launch_bounds__(kTileWaves * kWave) void k_merge_count(MergeParts mp, int32_t* __restrict__ cnt) {
  __shared__ uint32_t bits_s[kTileWaves][kMaxDenseD / 32];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  uint32_t* bits = bits_s[wave];
  const int wp = (int)((mp.d + 31) / 32);
  for (int64_t i = (int64_t)blockIdx.x * kTileWaves + wave; i < mp.n; i += (int64_t)gridDim.x * kTileWaves) {
    for (int w = lane; w < wp; w += kWave) bits[w] = 0u;
    wave_sync();
    for (int t = 0; t < mp.count; ++t)
      for (int p = mp.rp[t][i] + lane; p < mp.rp[t][i + 1]; p += kWave) {
        const int32_t c = mp.ci[t][p];
        if ((uint32_t)c < (uint64_t)mp.d) atomicOr(&bits[c >> 5], 1u << (c & 31));
      }
    wave_sync();
    int s = 0;
    for (int w = lane; w < wp; w += kWave) s += __popc(bits[w]);
    s = wave_sum_i32(s);
    if (lane == 0) cnt[i] = s;
    wave_sync();
  }
}

// Row sums: parts added in order into a d-wide FP64 strip, emitted in
// column order at the positions of out_rp.
__global__ __launch_bounds__(kTileWaves * kWave) void k_merge_values(MergeParts mp, const int32_t* __restrict__ out_rp,
                                                                     int32_t* __restrict__ out_ci,
                                                                     float* __restrict__ out_val) {
  __shared__ double strip_s[kTileWaves][kMaxDenseD];
  __shared__ uint32_t bits_s[kTileWaves][kMaxDenseD / 32];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  double* strip = strip_s[wave];
  uint32_t* bits = bits_s[wave];
  const int64_t d = mp.d;
  const int wp = (int)((d + 31) / 32);
  for (int64_t i = (int64_t)blockIdx.x * kTileWaves + wave; i < mp.n; i += (int64_t)gridDim.x * kTileWaves) {
    for (int w = lane; w < wp; w += kWave) bits[w] = 0u;
    for (int64_t c = lane; c < d; c += kWave) strip[c] = 0.0;
    wave_sync();
    for (int t = 0; t < mp.count; ++t) {  // parts in order; a part's columns are distinct
      for (int p = mp.rp[t][i] + lane; p < mp.rp[t][i + 1]; p += kWave) {
        const int32_t c = mp.ci[t][p];
        if ((uint32_t)c < (uint64_t)d) {
          strip[c] += (double)mp.val[t][p];
          atomicOr(&bits[c >> 5], 1u << (c & 31));
        }
      }
      wave_sync();
    }
    int64_t base = out_rp[i];
    for (int w0 = 0; w0 < wp; w0 += 2) {  // 64 columns at a time
      const uint64_t m = (uint64_t)bits[w0] | ((w0 + 1 < wp) ? (uint64_t)bits[w0 + 1] << 32 : 0ull);
      if ((m >> lane) & 1ull) {
        const int64_t pos = base + lanes_below(m);
        const int c = 32 * w0 + lane;
        out_ci[pos] = c;
        out_val[pos] = (float)strip[c];
      }
      base += __popcll(m);
    }
    wave_sync();
  }
}

static unsigned tile_grid(int64_t rows_per_wave_items) {
  const int64_t g = (rows_per_wave_items + kTileWaves - 1) / kTileWaves;
  return (unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

static int run_slice_count(const tsspgemm_csr* A, int32_t c0, int32_t c1, int32_t* out_rp, int64_t* nnz,
                           hipStream_t st) {
  int rc;
  if ((rc = check_csr(A, "A", false))) return rc;
  if (!out_rp || !nnz || c0 < 0 || c1 < c0) {
    set_error("column_slice: need out_rowptr, nnz and 0 <= c0 <= c1");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  const int64_t n = A->nrows;
  DevBuf cnt, scan;
  if ((rc = cnt.ensure((size_t)(n > 0 ? n : 1) * 4)) || (rc = scan.ensure((size_t)exscan_workspace_bytes(n))))
    return rc;
  if (n > 0) {
    k_slice_count<<<grid_for(n, 256) > 4096 ? 4096 : grid_for(n, 256), 256, 0, st>>>(n, A->rowptr, A->colidx, c0,
                                                                                    c1, (int32_t*)cnt.p);
    TSS_CHECK_LAUNCH();
  }
  if ((rc = launch_exscan_i32((const int32_t*)cnt.p, n, out_rp, (int64_t*)scan.p, st))) return rc;
  int32_t total = 0;
  TSS_HIP(hipMemcpyAsync(&total, out_rp + n, 4, hipMemcpyDeviceToHost, st));
  TSS_HIP(hipStreamSynchronize(st));
  *nnz = total;
  return TSSPGEMM_OK;
}

static int run_slice_fill(const tsspgemm_csr* A, int32_t c0, int32_t c1, const int32_t* out_rp, int32_t* out_ci,
                          float* out_val, hipStream_t st) {
  int rc;
  if ((rc = check_csr(A, "A", out_val != nullptr))) return rc;
  if (!out_rp || c0 < 0 || c1 < c0) {
    set_error("column_slice_fill: need out_rowptr and 0 <= c0 <= c1");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  const int64_t n = A->nrows;
  if (n == 0) return TSSPGEMM_OK;
  k_slice_fill<<<tile_grid(n), kTileWaves * kWave, 0, st>>>(n, A->rowptr, A->colidx, (const float*)A->vals, c0, c1,
                                                            out_rp, out_ci, out_val);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

static int make_parts(int32_t count, const tsspgemm_csr* parts, bool need_vals, MergeParts* mp) {
  if (count < 1 || !parts) {
    set_error("merge: need at least one part");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (count > kMergeMaxParts) {
    set_error("merge: more than 64 parts");
    return TSSPGEMM_ERR_UNSUPPORTED;
  }
  mp->count = count;
  mp->n = parts[0].nrows;
  mp->d = parts[0].ncols;
  for (int t = 0; t < count; ++t) {
    int rc;
    if ((rc = check_csr(&parts[t], "part", need_vals))) return rc;
    if (parts[t].nrows != mp->n || parts[t].ncols != mp->d) {
      set_error("merge: parts must all be n x d");
      return TSSPGEMM_ERR_INVALID_ARG;
    }
    mp->rp[t] = parts[t].rowptr;
    mp->ci[t] = parts[t].colidx;
    mp->val[t] = (const float*)parts[t].vals;
  }
  if (mp->d > kMaxDenseD) {
    set_error("merge: d > 1024");
    return TSSPGEMM_ERR_UNSUPPORTED;
  }
  return TSSPGEMM_OK;
}

static int run_merge_count(int32_t count, const tsspgemm_csr* parts, int32_t* out_rp, int64_t* nnz, hipStream_t st) {
  MergeParts mp{};
  int rc;
  if ((rc = make_parts(count, parts, false, &mp))) return rc;
  if (!out_rp || !nnz) {
    set_error("merge_count: need out_rowptr and nnz");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  const int64_t n = mp.n;
  DevBuf cnt, scan;
  if ((rc = cnt.ensure((size_t)(n > 0 ? n : 1) * 4)) || (rc = scan.ensure((size_t)exscan_workspace_bytes(n))))
    return rc;
  if (n > 0) {
    k_merge_count<<<tile_grid(n), kTileWaves * kWave, 0, st>>>(mp, (int32_t*)cnt.p);
    TSS_CHECK_LAUNCH();
  }
  if ((rc = launch_exscan_i32((const int32_t*)cnt.p, n, out_rp, (int64_t*)scan.p, st))) return rc;
  int32_t total = 0;
  TSS_HIP(hipMemcpyAsync(&total, out_rp + n, 4, hipMemcpyDeviceToHost, st));
  TSS_HIP(hipStreamSynchronize(st));
  *nnz = total;
  return TSSPGEMM_OK;
}

static int run_merge_values(int32_t count, const tsspgemm_csr* parts, const int32_t* out_rp, int32_t* out_ci,
                            float* out_val, hipStream_t st) {
  MergeParts mp{};
  int rc;
  if ((rc = make_parts(count, parts, true, &mp))) return rc;
  if (!out_rp || (mp.n > 0 && (!out_ci || !out_val))) {
    set_error("merge_values: need out_rowptr, out_colidx and out_vals");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (mp.n == 0) return TSSPGEMM_OK;
  k_merge_values<<<tile_grid(mp.n), kTileWaves * kWave, 0, st>>>(mp, out_rp, out_ci, out_val);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

}  // namespace tss

#define TSS_ABI_CALL(expr)                          \
  try {                                             \
    return (expr);                                  \
  } catch (...) {                                   \
    tss::set_error("unexpected C++ exception");     \
    return TSSPGEMM_ERR_HIP;                        \
  }

extern "C" int tsspgemm_column_slice_count(const tsspgemm_csr* A, int32_t c0, int32_t c1, int32_t* out_rowptr,
                                           int64_t* out_nnz, void* stream) {
  TSS_ABI_CALL(tss::run_slice_count(A, c0, c1, out_rowptr, out_nnz, (hipStream_t)stream))
}

extern "C" int tsspgemm_column_slice_fill(const tsspgemm_csr* A, int32_t c0, int32_t c1, const int32_t* out_rowptr,
                                          int32_t* out_colidx, float* out_vals, void* stream) {
  TSS_ABI_CALL(tss::run_slice_fill(A, c0, c1, out_rowptr, out_colidx, out_vals, (hipStream_t)stream))
}

extern "C" int tsspgemm_merge_count(int32_t count, const tsspgemm_csr* parts, int32_t* out_rowptr, int64_t* out_nnz,
                                    void* stream) {
  TSS_ABI_CALL(tss::run_merge_count(count, parts, out_rowptr, out_nnz, (hipStream_t)stream))
}

extern "C" int tsspgemm_merge_values(int32_t count, const tsspgemm_csr* parts, const int32_t* out_rowptr,
                                     int32_t* out_colidx, float* out_vals, void* stream) {
  TSS_ABI_CALL(tss::run_merge_values(count, parts, out_rowptr, out_colidx, out_vals, (hipStream_t)stream))
}
