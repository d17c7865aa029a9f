// CSR transpose of A's pattern: A^T row k lists the rows i with A(i,k) != 0 in
// ascending order, and perm gives each entry's position in A. This is the
// single-GPU form of the column-partitioned copy A^c that the paper keeps
// beside A (Sec. III-A); the backward pass uses it for dL/dB.
//
// Steps: column counts (atomics), exclusive scan into the row pointers,
// scatter of (i, p) pairs with per-column atomic cursors (order within a
// column then depends on timing), and a segmented sort of each transposed row
// by i (keys are distinct, so the result is unique): short segments by one
// thread, segments up to kSortTile by a workgroup bitonic sort in LDS, longer
// ones by sorting kSortTile-element tiles and merging runs pairwise.
#include "api_internal.hpp"

namespace tss {

constexpr int kSortTile = 4096;  // uint64 elements sorted in LDS by one workgroup (32 KB)
constexpr int kTinySeg = 16;

__global__ void k_col_count(int64_t nnz, const int32_t* __restrict__ aci, int32_t* __restrict__ cnt) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[aci[p]], 1);
}

// one thread per entry; its row comes from a binary search over the row
// pointers (an L2-resident array)
__global__ void k_scatter_t(int64_t n, int64_t nnz, const int32_t* __restrict__ arp, const int32_t* __restrict__ aci,
                            int32_t* __restrict__ cursor, uint64_t* __restrict__ pairs) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n;  // arp[lo] <= p < arp[hi]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (arp[mid] <= p) lo = mid; else hi = mid;
    }
    const int32_t q = atomicAdd(&cursor[aci[p]], 1);
    pairs[q] = ((uint64_t)(uint32_t)lo << 32) | (uint32_t)p;
  }
}

// short segments: insertion sort by one thread (in place, global memory)
__global__ void k_sort_tiny(int64_t m, const int32_t* __restrict__ trp, uint64_t* __restrict__ pairs) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int32_t a = trp[k], b = trp[k + 1];
  if (b - a < 2 || b - a > kTinySeg) return;
  for (int32_t x = a + 1; x < b; ++x) {
    const uint64_t v = pairs[x];
    int32_t y = x - 1;
    while (y >= a && pairs[y] > v) {
      pairs[y + 1] = pairs[y];
      --y;
    }
    pairs[y + 1] = v;
  }
}

// Bitonic sort of `len` (<= kSortTile) elements at `base`, by one workgroup.
__device__ void wg_sort_tile(uint64_t* base, int len, uint64_t* sh) {
  int p2 = 1;
  while (p2 < len) p2 <<= 1;
  for (int t = threadIdx.x; t < p2; t += blockDim.x) sh[t] = t < len ? base[t] : ~0ull;
  __syncthreads();
  for (int k = 2; k <= p2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < p2; t += blockDim.x) {
        const int u = t ^ j;
        if (u > t) {
          const bool up = (t & k) == 0;
          const uint64_t x = sh[t], y = sh[u];
          if ((x > y) == up) {
            sh[t] = y;
            sh[u] = x;
          }
        }
      }
      __syncthreads();
    }
  for (int t = threadIdx.x; t < len; t += blockDim.x) base[t] = sh[t];
  __syncthreads();
}

// segments with kTinySeg < len: sort tiles of kSortTile in LDS
__global__ __launch_bounds__(256) void k_sort_tiles(int64_t m, const int32_t* __restrict__ trp,
                                                    uint64_t* __restrict__ pairs) {
  __shared__ uint64_t sh[kSortTile];
  for (int64_t k = blockIdx.x; k < m; k += gridDim.x) {
    const int32_t a = trp[k], b = trp[k + 1];
    if (b - a <= kTinySeg) continue;
    for (int32_t t0 = a; t0 < b; t0 += kSortTile) wg_sort_tile(pairs + t0, min(kSortTile, b - t0), sh);
  }
}

// One merge pass over segments longer than `run`: adjacent sorted runs of
// length `run` are merged into runs of 2*run (src -> dst). Each thread places
// elements by rank (position in own run + lower/upper bound in the other run).
__global__ __launch_bounds__(256) void k_merge_pass(int64_t m, const int32_t* __restrict__ trp, int32_t run,
                                                    const uint64_t* __restrict__ src, uint64_t* __restrict__ dst) {
  for (int64_t k = blockIdx.x; k < m; k += gridDim.x) {
    const int32_t a = trp[k], b = trp[k + 1];
    const int32_t len = b - a;
    if (len <= kSortTile) continue;
    for (int32_t x = threadIdx.x; x < len; x += blockDim.x) {
      const int32_t pair0 = (x / (2 * run)) * (2 * run);
      const int32_t l0 = pair0, l1 = min(pair0 + run, len);
      const int32_t r0 = l1, r1 = min(pair0 + 2 * run, len);
      const uint64_t v = src[a + x];
      int32_t pos;
      if (x < l1) {  // element of the left run: count of right elements < v
        int32_t lo = r0, hi = r1;
        while (lo < hi) {
          const int32_t mid = (lo + hi) >> 1;
          if (src[a + mid] < v) lo = mid + 1; else hi = mid;
        }
        pos = pair0 + (x - l0) + (lo - r0);
      } else {  // element of the right run: count of left elements <= v (keys distinct)
        int32_t lo = l0, hi = l1;
        while (lo < hi) {
          const int32_t mid = (lo + hi) >> 1;
          if (src[a + mid] < v) lo = mid + 1; else hi = mid;
        }
        pos = pair0 + (x - r0) + (lo - l0);
      }
      dst[a + pos] = v;
    }
  }
}

__global__ void k_unpack_t(int64_t nnz, const uint64_t* __restrict__ pairs, int32_t* __restrict__ tci,
                           int32_t* __restrict__ perm) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t v = pairs[q];
    tci[q] = (int32_t)(v >> 32);
    perm[q] = (int32_t)(uint32_t)v;
  }
}

__global__ void k_max_seg(int64_t m, const int32_t* __restrict__ trp, int32_t* __restrict__ out) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < m) atomicMax(out, trp[k + 1] - trp[k]);
}

static int run_transpose(const tsspgemm_csr* A, int32_t* trp, int32_t* tci, int32_t* perm, hipStream_t st) {
  int rc;
  if ((rc = check_csr(A, "A", false))) return rc;
  if (!trp || (A->nnz > 0 && (!tci || !perm))) {
    set_error("transpose: NULL output");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  const int64_t n = A->nrows, m = A->ncols, nnz = A->nnz;
  DevBuf cnt, cursor, pairs, tmp, mx, scan;
  if ((rc = cnt.ensure((size_t)(m + 1) * 4)) || (rc = cursor.ensure((size_t)(m + 1) * 4)) ||
      (rc = scan.ensure((size_t)exscan_workspace_bytes(m))) ||
      (rc = pairs.ensure((size_t)(nnz + 1) * 8)) || (rc = tmp.ensure((size_t)(nnz + 1) * 8)) || (rc = mx.ensure(4)))
    return rc;
  if ((rc = launch_zero_bytes(cnt.p, (size_t)(m + 1) * 4, st)) || (rc = launch_zero_bytes(mx.p, 4, st))) return rc;
  if (nnz > 0) k_col_count<<<grid_for(nnz, 256 * 4) > 8192 ? 8192 : grid_for(nnz, 256 * 4), 256, 0, st>>>(
      nnz, A->colidx, (int32_t*)cnt.p);
  TSS_CHECK_LAUNCH();
  if ((rc = launch_exscan_i32((const int32_t*)cnt.p, m, trp, (int64_t*)scan.p, st))) return rc;
  TSS_HIP(hipMemcpyAsync(cursor.p, trp, (size_t)m * 4, hipMemcpyDeviceToDevice, st));
  if (nnz > 0) k_scatter_t<<<grid_for(nnz, 256) > 65536 ? 65536 : grid_for(nnz, 256), 256, 0, st>>>(
      n, nnz, A->rowptr, A->colidx, (int32_t*)cursor.p, (uint64_t*)pairs.p);
  if (m > 0) {
    k_sort_tiny<<<grid_for(m, 256), 256, 0, st>>>(m, trp, (uint64_t*)pairs.p);
    k_sort_tiles<<<(unsigned)(m < 8192 ? m : 8192), 256, 0, st>>>(m, trp, (uint64_t*)pairs.p);
    k_max_seg<<<grid_for(m, 256), 256, 0, st>>>(m, trp, (int32_t*)mx.p);
  }
  TSS_CHECK_LAUNCH();
  int32_t longest = 0;
  TSS_HIP(hipMemcpyAsync(&longest, mx.p, 4, hipMemcpyDeviceToHost, st));
  TSS_HIP(hipStreamSynchronize(st));
  uint64_t* src = (uint64_t*)pairs.p;
  uint64_t* dst = (uint64_t*)tmp.p;
  if (longest > kSortTile) {
    // segments below the cut keep their data in `src`; copy it along so that
    // the final buffer is complete whichever buffer the passes end in
    TSS_HIP(hipMemcpyAsync(dst, src, (size_t)nnz * 8, hipMemcpyDeviceToDevice, st));
    for (int32_t run = kSortTile; run < longest; run *= 2) {
      k_merge_pass<<<(unsigned)(m < 8192 ? m : 8192), 256, 0, st>>>(m, trp, run, src, dst);
      TSS_CHECK_LAUNCH();
      uint64_t* t = src;
      src = dst;
      dst = t;
    }
  }
  if (nnz > 0) k_unpack_t<<<grid_for(nnz, 256 * 4) > 8192 ? 8192 : grid_for(nnz, 256 * 4), 256, 0, st>>>(
      nnz, src, tci, perm);
  TSS_CHECK_LAUNCH();
  TSS_HIP(hipStreamSynchronize(st));  // the temporary buffers are released on return
  return TSSPGEMM_OK;
}

}  // namespace tss

extern "C" int tsspgemm_transpose(const tsspgemm_csr* A, int32_t* at_rowptr, int32_t* at_colidx, int32_t* at_perm,
                                  void* stream) {
  try {
    return tss::run_transpose(A, at_rowptr, at_colidx, at_perm, (hipStream_t)stream);
  } catch (...) {
    tss::set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}
