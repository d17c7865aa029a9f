// CSR transpose of A's pattern: A^T row k lists the rows i with A(i,k) != 0 in
// ascending order, and perm gives each entry's position in A. This is the
// single-GPU form of the column-partitioned copy A^c that the paper keeps
// beside A (Sec. III-A); the backward pass uses it for dL/dB.
//
// A's entries are already in row order, so a stable sort of the entry
// positions by column gives A^T directly (within a column the rows stay
// ascending). The sort is a least-significant-digit radix sort with 8-bit
// digits over the column index (ceil(log2(ncols) / 8) passes). Each pass:
// per-tile digit histograms (4096 entries a tile), one exclusive scan over
// them in digit-major order, then a scatter in which every tile ranks its
// entries stably (entries in index order; within a wavefront, lanes with the
// same digit are found with eight ballots). Afterwards the row pointers come
// from the column boundaries of the sorted keys, and each entry's row from a
// binary search over A's row pointers (in entry order), gathered through the
// permutation. Deterministic, no atomics on global memory.
#include "api_internal.hpp"

namespace tss {

constexpr int kRsThreads = 256;
constexpr int kRsPer = 16;                        // entries per thread per tile
constexpr int kRsTile = kRsThreads * kRsPer;      // 4096
constexpr int kRsDigits = 256;

// hist[digit * ntiles + tile] = entries of the tile whose key has that digit
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(int64_t nnz, const int32_t* __restrict__ keys, int shift,
                                                        int64_t ntiles, int32_t* __restrict__ hist) {
  __shared__ int32_t h[kRsDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
  for (int r = 0; r < kRsPer; ++r) {
    const int64_t e = base + r * kRsThreads + threadIdx.x;
    if (e < nnz) atomicAdd(&h[(keys[e] >> shift) & (kRsDigits - 1)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile. Entries are taken in rounds of 256 (index
// order); an entry's destination is its digit's offset for this tile, plus
// the entries with the same digit in earlier rounds, in earlier wavefronts of
// this round, and in lower lanes of its wavefront.
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(int64_t nnz, const int32_t* __restrict__ keys_in,
                                                           const int32_t* __restrict__ vals_in, int shift,
                                                           int64_t ntiles, const int32_t* __restrict__ offs,
                                                           int32_t* __restrict__ keys_out,
                                                           int32_t* __restrict__ vals_out) {
  __shared__ int32_t base_s[kRsDigits];                 // offset of each digit for this tile, advanced per round
  __shared__ int32_t wcnt[kRsThreads / kWave][kRsDigits];  // per-wavefront digit counts of the round
  const int wave = threadIdx.x >> 6;
  base_s[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
  const int64_t tile0 = (int64_t)blockIdx.x * kRsTile;
  for (int r = 0; r < kRsPer; ++r) {
    for (int w = 0; w < kRsThreads / kWave; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t e = tile0 + r * kRsThreads + threadIdx.x;
    const bool valid = e < nnz;
    int32_t key = 0, val = 0;
    if (valid) {
      key = keys_in[e];
      val = vals_in ? vals_in[e] : (int32_t)e;
    }
    const int dg = (key >> shift) & (kRsDigits - 1);
    // lanes of this wavefront holding the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t ones = __ballot(valid && ((dg >> bit) & 1));
      peers &= ((dg >> bit) & 1) ? ones : ~ones;
    }
    const int below = lanes_below(peers);
    if (valid && below == 0) wcnt[wave][dg] = __popcll(peers);  // the lowest peer reports the count
    __syncthreads();
    if (valid) {
      int pos = base_s[dg] + below;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][dg];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    int add = 0;
    for (int w = 0; w < kRsThreads / kWave; ++w) add += wcnt[w][threadIdx.x];
    base_s[threadIdx.x] += add;
    __syncthreads();
  }
}

// trp[c] = first position of column c in the sorted keys (trp[m] = nnz):
// each boundary between different keys fills the pointers of the columns
// it skips over.
__global__ void k_col_bounds(int64_t nnz, int64_t m, const int32_t* __restrict__ keys, int32_t* __restrict__ trp) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x <= nnz; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lo = x == 0 ? 0 : (int64_t)keys[x - 1] + 1;  // columns whose first position is x
    const int64_t hi = x == nnz ? m : (int64_t)keys[x];
    for (int64_t c = lo; c <= hi && c <= m; ++c) trp[c] = (int32_t)x;
  }
}

// rowof[p] = row of A entry p: a binary search over A's row pointers, in
// entry order (neighbouring threads take the same path through the search)
__global__ void k_rows_of(int64_t n, int64_t nnz, const int32_t* __restrict__ arp, int32_t* __restrict__ rowof) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n;  // arp[lo] <= p < arp[hi]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (arp[mid] <= p)
        lo = mid;
      else
        hi = mid;
    }
    rowof[p] = (int32_t)lo;
  }
}

// tci[x] = rowof[perm[x]]
__global__ void k_gather_rows(int64_t nnz, const int32_t* __restrict__ perm, const int32_t* __restrict__ rowof,
                              int32_t* __restrict__ tci) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nnz; x += (int64_t)gridDim.x * blockDim.x)
    tci[x] = rowof[perm[x]];
}

static int run_transpose(const tsspgemm_csr* A, int32_t* trp, int32_t* tci, int32_t* perm, hipStream_t st) {
  int rc;
  if ((rc = check_csr(A, "A", false))) return rc;
  if (!trp || (A->nnz > 0 && (!tci || !perm))) {
    set_error("transpose: NULL output");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  const int64_t n = A->nrows, m = A->ncols, nnz = A->nnz;
  if (nnz == 0) {
    if ((rc = launch_fill_i32(trp, m + 1, 0, st))) return rc;
    TSS_HIP(hipStreamSynchronize(st));
    return TSSPGEMM_OK;
  }
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < m) ++bits;
  const int passes = (bits + 7) / 8;
  const int64_t ntiles = (nnz + kRsTile - 1) / kRsTile;
  const int64_t nh = ntiles * kRsDigits;
  DevBuf k0, v0, k1, v1, hist, offs, scan;
  if ((rc = k0.ensure((size_t)nnz * 4)) || (rc = v0.ensure((size_t)nnz * 4)) || (rc = k1.ensure((size_t)nnz * 4)) ||
      (rc = v1.ensure((size_t)nnz * 4)) || (rc = hist.ensure((size_t)nh * 4)) ||
      (rc = offs.ensure((size_t)(nh + 1) * 4)) || (rc = scan.ensure((size_t)exscan_workspace_bytes(nh))))
    return rc;
  const int32_t* kin = A->colidx;  // pass 0 reads A's columns, values = positions
  const int32_t* vin = nullptr;
  int32_t* kout = (int32_t*)k0.p;
  int32_t* vout = (int32_t*)v0.p;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 8 * pass;
    k_rs_hist<<<(unsigned)ntiles, kRsThreads, 0, st>>>(nnz, kin, shift, ntiles, (int32_t*)hist.p);
    TSS_CHECK_LAUNCH();
    if ((rc = launch_exscan_i32((const int32_t*)hist.p, nh, (int32_t*)offs.p, (int64_t*)scan.p, st))) return rc;
    k_rs_scatter<<<(unsigned)ntiles, kRsThreads, 0, st>>>(nnz, kin, vin, shift, ntiles, (const int32_t*)offs.p,
                                                          kout, vout);
    TSS_CHECK_LAUNCH();
    kin = kout;
    vin = vout;
    kout = (kout == (int32_t*)k0.p) ? (int32_t*)k1.p : (int32_t*)k0.p;
    vout = (vout == (int32_t*)v0.p) ? (int32_t*)v1.p : (int32_t*)v0.p;
  }
  // kin / vin: keys (columns) and A positions in A^T order
  const unsigned g = grid_for(nnz + 1, 256) > 8192 ? 8192 : grid_for(nnz + 1, 256);
  k_col_bounds<<<g, 256, 0, st>>>(nnz, m, kin, trp);
  TSS_HIP(hipMemcpyAsync(perm, vin, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st));
  int32_t* rowof = kout;  // the keys buffer the last pass did not write
  k_rows_of<<<g, 256, 0, st>>>(n, nnz, A->rowptr, rowof);
  k_gather_rows<<<g, 256, 0, st>>>(nnz, vin, rowof, tci);
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
