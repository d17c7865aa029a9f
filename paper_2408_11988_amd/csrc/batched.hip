// Batched plus-times TS-SpGEMM: many independent products C_t = A_t B_t of
// uneven n, d and density, each phase one launch over all instances.
//
// A batch plan keeps, in device memory, one descriptor per instance (its
// arrays, its slices of the batch workspace, its work-class thresholds) and
// prefix sums of per-instance block counts; a kernel finds its instance by
// binary search over those prefix sums. Work items of all instances share one
// binned list ordered heaviest first, so the persistent numeric kernels
// balance across instances. The output pool offsets of the instances come
// from a device-side scan over the instances' nnz, so a run needs no host
// synchronisation and no allocation and can be captured in a HIP graph
// (tsspgemm_batched_capture / tsspgemm_batched_launch).
#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include "api_internal.hpp"
#include "dev_numeric.hpp"
#include "dev_symbolic.hpp"

namespace tss {

struct BInst {
  Problem pr;  // crp / cci / cval are set on the device by k_b_scan
  NumThresholds th;
  int32_t* cnt;    // nnz of each C row (workspace)
  int64_t rp_off;  // start of the instance's row pointers in the caller's array
  int32_t gl;      // lanes per B row in the wavefront / workgroup kernel (64 for flat products)
  int32_t lgl;     // lanes per row group in the light kernel
  int32_t flat;    // product layout: kLayoutRows, kLayoutFlat or kLayoutVec
  int32_t rank;    // place of the instance in the numeric work list (instances of one launch class are adjacent)
};

struct BatchDev {
  BInst* insts;
  int32_t count;
  int32_t dmax;
  int32_t sym_split;
  int32_t idb;  // bytes of the narrowed B column ids (1: dmax <= 256, else 2)
  int32_t r_lo, r_hi;  // per-class launches: the ranks of the instances this launch runs
  int32_t lds_d, pad2;  // numeric launches: strip stride in LDS (largest d of the class)
  const int64_t* row_off;  // prefix sums over instances: rows
  const int64_t* bm_off;   // bitmap blocks (kBmRows rows)
  const int64_t* rrow_off;  // rows of the instances in rank order: prefix sums (count + 1)
  const int64_t* rank_t;    // the instance of each rank
  const int64_t* sb_off;   // scan blocks (kScanRows rows)
  int64_t total_rows, total_sb;
  Item* sym_items;
  int32_t* sym_inst;
  Item* num_items;
  int32_t* num_inst;
  SplitRow* split_rows;  // pad = instance
  double* partial;       // slot x dmax
  int64_t* block_sums;   // [total_sb] nnz sums, then [total_sb] product sums
  int64_t* inst_flops;   // products per instance
  int32_t* nb_cnt;       // numeric work list: items per key (class, instance, bin), then
  int32_t* nb_cur;       //   the fill counter and
  int32_t* nb_off;       //   the offset of each key (kNumClasses x count x kBins each, then the total)
  int32_t* sb_cnt;       // symbolic work list: items per key (instance, bin), the fill
  int32_t* sb_cur;       //   counter and the offset of each key (count x kBins each)
  int32_t* sb_kof;
  Counters* ctr;
  int32_t* c_rowptrs;  // run outputs
  int32_t* pool_ci;
  float* pool_val;
  int64_t* c_off;
};

__device__ __forceinline__ int find_inst(const int64_t* off, int count, int64_t x) {
  int lo = 0, hi = count;  // off[lo] <= x < off[hi]; empty instances are skipped
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// The rank r in [lo, hi) with off[r] <= x < off[r + 1].
__device__ __forceinline__ int find_rank(const int64_t* off, int lo, int hi, int64_t x) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

constexpr int32_t kBatchSymSplit = 2048;  // symbolic split size of a batch without tunings

// Each A entry's B row bounds (brp[k], brp[k + 1]) for its column k, built
// once by the batch plan (the patterns are fixed for the batch's life) and
// read by the numeric staging instead of gathering B's row pointers.
__global__ void k_b_entry_bounds(const int32_t* __restrict__ aci, const int32_t* __restrict__ brp, int64_t nnz,
                                 int2* __restrict__ out) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    const int k = aci[p];
    out[p] = make_int2(brp[k], brp[k + 1]);
  }
}

__global__ void k_b_zero(Counters* ctr) {
  uint32_t* p = (uint32_t*)ctr;
  for (size_t t = threadIdx.x; t < sizeof(Counters) / 4; t += blockDim.x) p[t] = 0u;
}

__global__ __launch_bounds__(256) void k_b_bitmap(BatchDev b) {
  extern __shared__ __align__(16) uint32_t sm[];
  const int t = find_inst(b.bm_off, b.count, blockIdx.x);
  const Problem& pr = b.insts[t].pr;
  bitmap_block(pr.n, pr.brp, pr.bci, pr.wp, (uint32_t*)pr.bbits, (int64_t)(blockIdx.x - b.bm_off[t]) * kBmRows, sm,
               b.idb == 1 ? (uint8_t*)pr.bcol : nullptr, b.idb == 2 ? (uint16_t*)pr.bcol : nullptr);
}

// ---------------------------------------------------------------- symbolic

// The symbolic work list (rows with more A entries than a light slot takes,
// and chunks of split rows) is ordered by instance rank, then heaviest bin
// first: key (rank, bin), so the wavefronts running at one time gather the B
// bitmap rows of one or two instances, and the instances of one bitmap width
// (adjacent ranks) hold one contiguous range. A workgroup takes kScanRows
// rows of one instance (the scan blocks, sb_off).
__global__ void k_b_sym_bin_count(BatchDev b) {
  __shared__ int32_t hist[kBins];
  if (threadIdx.x < kBins) hist[threadIdx.x] = 0;
  __syncthreads();
  const int t = find_inst(b.sb_off, b.count, blockIdx.x);
  const Problem& pr = b.insts[t].pr;
  const int64_t r0 = (blockIdx.x - b.sb_off[t]) * (int64_t)kScanRows;
  const int64_t r1 = min((int64_t)pr.n, r0 + kScanRows);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    int bin, count;
    sym_bin(pr.arp[i + 1] - pr.arp[i], b.sym_split, bin, count);
    if (count) atomicAdd(&hist[bin], count);
  }
  __syncthreads();
  if (threadIdx.x < kBins && hist[threadIdx.x])
    atomicAdd(&b.sb_cnt[b.insts[t].rank * kBins + threadIdx.x], hist[threadIdx.x]);
}

// One workgroup: exclusive scan of the (instance, bin) counts into offsets,
// and the item total.
__global__ __launch_bounds__(kScanThreads) void k_b_sym_bin_scan(BatchDev b) {
  __shared__ long long sh[32];
  const int64_t nk = (int64_t)b.count * kBins;
  long long carry = 0;
  for (int64_t x0 = 0; x0 < nk; x0 += kScanThreads) {
    const int64_t x = x0 + threadIdx.x;
    const long long v = x < nk ? b.sb_cnt[x] : 0;
    long long tot;
    const long long ex = block_exscan_1024(v, sh, &tot);
    if (x < nk) b.sb_kof[x] = (int32_t)(carry + ex);
    carry += tot;
  }
  if (threadIdx.x == 0) {
    b.sb_kof[nk] = (int32_t)carry;
    b.ctr->sym_total = (int32_t)carry;
  }
}

__global__ void k_b_sym_bin_fill(BatchDev b) {
  __shared__ int32_t cnt[kBins], base[kBins];
  if (threadIdx.x < kBins) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int t = find_inst(b.sb_off, b.count, blockIdx.x);
  const Problem& pr = b.insts[t].pr;
  const int64_t r0 = (blockIdx.x - b.sb_off[t]) * (int64_t)kScanRows;
  const int64_t r1 = min((int64_t)pr.n, r0 + kScanRows);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {  // counts of this workgroup's rows
    int bin, count;
    sym_bin(pr.arp[i + 1] - pr.arp[i], b.sym_split, bin, count);
    if (count) atomicAdd(&cnt[bin], count);
  }
  __syncthreads();
  if (threadIdx.x < kBins) {
    if (cnt[threadIdx.x]) {
      const int k = b.insts[t].rank * kBins + threadIdx.x;
      base[threadIdx.x] = b.sb_kof[k] + atomicAdd(&b.sb_cur[k], cnt[threadIdx.x]);
    }
    cnt[threadIdx.x] = 0;
  }
  __syncthreads();
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const int a = pr.arp[i], m = pr.arp[i + 1] - a;
    int bin, count;
    sym_bin(m, b.sym_split, bin, count);
    if (!count) continue;
    const int pos = base[bin] + atomicAdd(&cnt[bin], count);
    if (m <= b.sym_split) {
      b.sym_items[pos] = Item{(int32_t)i, a, a + m, 0};
      b.sym_inst[pos] = t;
    } else {
      for (int c = 0; c < count; ++c) {
        const int p0 = a + c * b.sym_split;
        b.sym_items[pos + c] = Item{(int32_t)i, p0, min(a + m, p0 + b.sym_split), kSplitFlag | c};
        b.sym_inst[pos + c] = t;
      }
    }
  }
}

__global__ void k_b_sym_split_zero(BatchDev b) {
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x >= b.ctr->sym_total) return;
  const Item it = b.sym_items[x];
  if ((it.aux & kSplitFlag) == 0 || (it.aux & ~kSplitFlag) != 0) return;
  const Problem& pr = b.insts[b.sym_inst[x]].pr;
  for (int w = 0; w < pr.wp; ++w) pr.cbits[(int64_t)it.row * pr.wp + w] = 0u;
  pr.flops[it.row] = 0;
}

// The symbolic kernels run once per bitmap width: the instances of ranks
// [r_lo, r_hi) share it. Light rows are numbered in rank order (rrow_off).

// Bitmaps of at most 8 words: a lane owns a light row and ORs whole B
// bitmap rows (16-byte loads), as in the single-product pass.
template <int WP>
__global__ __launch_bounds__(kBlock) void k_b_sym_light_lanes(BatchDev b) {
  const int64_t x_end = b.rrow_off[b.r_hi];
  // the wavefront's first row, and its rank found once for the wavefront
  // (wave-uniform); lanes past the rank's last row (a wavefront that spans
  // two instances) search on from the next rank
  const int64_t xw = b.rrow_off[b.r_lo] + (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1));
  if (xw >= x_end) return;
  int r = __builtin_amdgcn_readfirstlane(find_rank(b.rrow_off, b.r_lo, b.r_hi, xw));
  const int64_t x = xw + (threadIdx.x & (kWave - 1));
  if (x >= x_end) return;
  if (x >= b.rrow_off[r + 1]) r = find_rank(b.rrow_off, r + 1, b.r_hi, x);
  const Problem& pr = b.insts[b.rank_t[r]].pr;
  const int64_t row = x - b.rrow_off[r];
  const int p0 = pr.arp[row], p1 = pr.arp[row + 1];
  if (p1 - p0 > kSlotRowMax) return;  // a heavy row: done from the item list
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

// Heavy rows and split chunks of ranks [r_lo, r_hi): a wavefront per item,
// a lane per A entry (whole B bitmap rows), OR-ed across the wavefront.
template <int WP>
__global__ __launch_bounds__(kBlock) void k_b_symbolic_lanes(BatchDev b) {
  const int lane = threadIdx.x & (kWave - 1);
  const int x0 = b.sb_kof[b.r_lo * kBins], x1 = b.sb_kof[b.r_hi * kBins];
  for (int x = x0 + blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); x < x1; x += gridDim.x * kWavesPerBlock) {
    const Item it = b.sym_items[x];
    const Problem& pr = b.insts[b.sym_inst[x]].pr;
    const bool split = (it.aux & kSplitFlag) != 0;
    int fl = 0;
    const uint32_t word = sym_item_or<WP>(pr, it.p0, it.p1, lane, fl);
    const long long fsum = (int64_t)(it.p1 - it.p0) * 32 * WP < (1ll << 31) ? (long long)wave_sum_i32(fl)
                                                                              : wave_sum_i64((long long)fl);
    if ((lane & (kWave / WP - 1)) == 0) {  // the first lane holding each word
      uint32_t* dst = &pr.cbits[(int64_t)it.row * WP + bm_word_of<WP>(lane)];
      if (split) {
        if (word) atomicOr(dst, word);
      } else {
        *dst = word;
      }
    }
    if (lane == 0) {
      if (split)
        atomicAdd((unsigned long long*)&pr.flops[it.row], (unsigned long long)fsum);
      else
        pr.flops[it.row] = fsum;
    }
  }
}

// Wider bitmaps (16 or 32 words): a slot of wp lanes per light row, a lane
// per word.
__global__ __launch_bounds__(kBlock) void k_b_sym_light(BatchDev b, int wp) {
  const int ns = kWave / wp;
  const int lane = threadIdx.x & (kWave - 1);
  const int slot = lane / wp, w = lane & (wp - 1);
  const int64_t gw = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int64_t x = b.rrow_off[b.r_lo] + gw * ns + slot;
  if (x >= b.rrow_off[b.r_hi]) return;
  const int r = find_rank(b.rrow_off, b.r_lo, b.r_hi, x);
  const Problem& pr = b.insts[b.rank_t[r]].pr;
  const int64_t row = x - b.rrow_off[r];
  const int p0 = pr.arp[row], p1 = pr.arp[row + 1];
  if (p1 - p0 > kSlotRowMax) return;
  uint32_t acc = 0u;
  int fl = 0;
  int p = p0;
  for (; p + 3 < p1; p += 4) {
    const int k0 = pr.aci[p], k1 = pr.aci[p + 1], k2 = pr.aci[p + 2], k3 = pr.aci[p + 3];
    const uint32_t x0 = pr.bbits[(int64_t)k0 * wp + w], x1 = pr.bbits[(int64_t)k1 * wp + w];
    const uint32_t x2 = pr.bbits[(int64_t)k2 * wp + w], x3 = pr.bbits[(int64_t)k3 * wp + w];
    acc |= (x0 | x1) | (x2 | x3);
    fl += __popc(x0) + __popc(x1) + __popc(x2) + __popc(x3);
  }
  for (; p < p1; ++p) {
    const uint32_t v = pr.bbits[(int64_t)pr.aci[p] * wp + w];
    acc |= v;
    fl += __popc(v);
  }
  for (int o = 1; o < wp; o <<= 1) fl += __shfl_xor(fl, o, kWave);
  pr.cbits[row * wp + w] = acc;
  if (w == 0) pr.flops[row] = fl;
}

// Wider bitmaps: heavy rows and split chunks, a wavefront per item, a slot
// of wp lanes per A entry.
__global__ __launch_bounds__(kBlock) void k_b_symbolic(BatchDev b, int wp) {
  const int lane = threadIdx.x & (kWave - 1);
  const int slot = lane / wp, w = lane & (wp - 1);
  const int x0 = b.sb_kof[b.r_lo * kBins], x1 = b.sb_kof[b.r_hi * kBins];
  for (int x = x0 + blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); x < x1; x += gridDim.x * kWavesPerBlock) {
    const Item it = b.sym_items[x];
    const Problem& pr = b.insts[b.sym_inst[x]].pr;
    const bool split = (it.aux & kSplitFlag) != 0;
    int fl = 0;
    uint32_t acc = sym_item_or_slots(pr, it.p0, it.p1, wp, lane, word_cols(pr.d, w), fl);
    for (int o = wp; o < kWave; o <<= 1) acc |= shfl_xor_u32(acc, o);
    const long long fsum = wave_sum_i64((long long)fl);
    if (slot == 0) {
      if (split) {
        if (acc) atomicOr(&pr.cbits[(int64_t)it.row * wp + w], acc);
      } else {
        pr.cbits[(int64_t)it.row * wp + w] = acc;
      }
    }
    if (lane == 0) {
      if (split)
        atomicAdd((unsigned long long*)&pr.flops[it.row], (unsigned long long)fsum);
      else
        pr.flops[it.row] = fsum;
    }
  }
}

// ---------------------------------------------------------------- counts and scans

__global__ __launch_bounds__(kScanThreads) void k_b_count_rows(BatchDev b) {
  __shared__ long long sh[32];
  const int t = find_inst(b.sb_off, b.count, blockIdx.x);
  const BInst& in = b.insts[t];
  const Problem& pr = in.pr;
  const int64_t base = (blockIdx.x - b.sb_off[t]) * (int64_t)kScanRows;
  long long s = 0, f = 0;
  for (int u = 0; u < kScanPer; ++u) {
    const int64_t i = base + u * kScanThreads + threadIdx.x;
    if (i < pr.n) {
      int c = 0;
      for (int w = 0; w < pr.wp; ++w) c += __popc(pr.cbits[i * pr.wp + w]);
      in.cnt[i] = c;
      s += c;
      f += pr.flops[i];
    }
  }
  long long tot, ftot;
  block_exscan_1024(s, sh, &tot);
  block_exscan_1024(f, sh, &ftot);
  if (threadIdx.x == 0) {
    b.block_sums[blockIdx.x] = tot;
    b.block_sums[b.total_sb + blockIdx.x] = ftot;
  }
}

// One workgroup: an exclusive scan of the block sums of all instances in
// order (nnz and products). An instance's C pool offset is the scan at its
// first block; k_b_write_rowptr subtracts it to get offsets inside the
// instance. Also sets every instance's C pointers into the pools.
__global__ __launch_bounds__(kScanThreads) void k_b_scan(BatchDev b) {
  __shared__ long long sh[32];
  long long carry = 0, fcarry = 0;
  for (int64_t x0 = 0; x0 < b.total_sb; x0 += kScanThreads) {
    const int64_t x = x0 + threadIdx.x;
    const long long v = x < b.total_sb ? b.block_sums[x] : 0;
    const long long f = x < b.total_sb ? b.block_sums[b.total_sb + x] : 0;
    long long tot, ftot;
    const long long ex = block_exscan_1024(v, sh, &tot);
    const long long fex = block_exscan_1024(f, sh, &ftot);
    if (x < b.total_sb) {
      b.block_sums[x] = carry + ex;
      b.block_sums[b.total_sb + x] = fcarry + fex;
    }
    carry += tot;
    fcarry += ftot;
  }
  __syncthreads();  // the scanned sums are read back below by other threads
  for (int t = threadIdx.x; t < b.count; t += kScanThreads) {
    const int64_t s0 = b.sb_off[t], s1 = b.sb_off[t + 1];
    const long long pool = s0 < b.total_sb ? b.block_sums[s0] : carry;
    const long long f0 = s0 < b.total_sb ? b.block_sums[b.total_sb + s0] : fcarry;
    const long long f1 = s1 < b.total_sb ? b.block_sums[b.total_sb + s1] : fcarry;
    BInst& in = b.insts[t];
    b.c_off[t] = pool;
    b.inst_flops[t] = f1 - f0;
    in.pr.crp = b.c_rowptrs ? b.c_rowptrs + in.rp_off : nullptr;
    in.pr.cci = b.pool_ci ? b.pool_ci + pool : nullptr;
    in.pr.cval = b.pool_val ? (void*)(b.pool_val + pool) : nullptr;
  }
  if (threadIdx.x == 0) {
    b.c_off[b.count] = carry;
    b.ctr->nnz_total = carry;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_b_write_rowptr(BatchDev b) {
  __shared__ long long sh[32];
  const int t = find_inst(b.sb_off, b.count, blockIdx.x);
  const BInst& in = b.insts[t];
  const int64_t n = in.pr.n;
  int32_t* crp = b.c_rowptrs + in.rp_off;
  const int64_t base = (blockIdx.x - b.sb_off[t]) * (int64_t)kScanRows;
  long long carry = b.block_sums[blockIdx.x] - b.c_off[t];  // offset inside instance t
  for (int u = 0; u < kScanPer; ++u) {
    const int64_t i = base + u * kScanThreads + threadIdx.x;
    const long long v = i < n ? in.cnt[i] : 0;
    long long tot;
    const long long ex = block_exscan_1024(v, sh, &tot);
    if (i < n) crp[i] = (int32_t)(carry + ex);
    if (i == n - 1) crp[n] = (int32_t)(carry + ex + v);
    carry += tot;
  }
}

// instances without rows still get rowptr[0] = 0
__global__ void k_b_empty_rowptr(BatchDev b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < b.count && b.insts[t].pr.n == 0) b.c_rowptrs[b.insts[t].rp_off] = 0;
}

// ---------------------------------------------------------------- numeric binning

// The work list is ordered by class, then by instance rank, then heaviest
// bin first: key (cls, rank, bin). The numeric launches walk it in order, so
// the wavefronts running at one time gather B rows of one or two instances
// (whose B fits the caches) rather than of every instance of the batch, and
// the instances of one launch class (ranks [r_lo, r_hi)) hold one contiguous
// range of each class. A workgroup takes kScanRows rows of one instance (the
// scan blocks, sb_off).
__device__ __forceinline__ int nb_key(const BatchDev& b, int cls, int rank, int bin) {
  return (cls * b.count + rank) * kBins + bin;
}

// Items of class cls of this launch's instances: [lo, hi) of the work list.
__device__ __forceinline__ int2 nb_range(const BatchDev& b, int cls) {
  return make_int2(b.nb_off[nb_key(b, cls, b.r_lo, 0)], b.nb_off[nb_key(b, cls, b.r_hi, 0)]);
}

__global__ void k_b_num_bin_count(BatchDev b) {
  __shared__ int32_t hist[kNumClasses * kBins];
  for (int x = threadIdx.x; x < kNumClasses * kBins; x += blockDim.x) hist[x] = 0;
  __syncthreads();
  const int t = find_inst(b.sb_off, b.count, blockIdx.x);
  const BInst& in = b.insts[t];
  const int64_t r0 = (blockIdx.x - b.sb_off[t]) * (int64_t)kScanRows;
  const int64_t r1 = min((int64_t)in.pr.n, r0 + kScanRows);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const int64_t f = in.pr.flops[i];
    if (f > 0) {
      int cls, key, count, ce;
      num_key(f, in.pr.arp[i + 1] - in.pr.arp[i], in.th, cls, key, count, ce);
      atomicAdd(&hist[key], count);
    }
  }
  __syncthreads();
  for (int x = threadIdx.x; x < kNumClasses * kBins; x += blockDim.x)
    if (hist[x]) atomicAdd(&b.nb_cnt[nb_key(b, x / kBins, in.rank, x % kBins)], hist[x]);
}

// One workgroup: exclusive scan of the key counts into the key offsets, and
// the class totals.
__global__ __launch_bounds__(kScanThreads) void k_b_num_bin_scan(BatchDev b) {
  __shared__ long long sh[32];
  const int64_t nk = (int64_t)kNumClasses * b.count * kBins;
  long long carry = 0;
  for (int64_t x0 = 0; x0 < nk; x0 += kScanThreads) {
    const int64_t x = x0 + threadIdx.x;
    const long long v = x < nk ? b.nb_cnt[x] : 0;
    long long tot;
    const long long ex = block_exscan_1024(v, sh, &tot);
    if (x < nk) b.nb_off[x] = (int32_t)(carry + ex);
    carry += tot;
  }
  if (threadIdx.x == 0) b.nb_off[nk] = (int32_t)carry;
  __syncthreads();  // the offsets are read back below by other threads
  if (threadIdx.x < kNumClasses) {
    const int c = threadIdx.x;
    const int64_t x0 = (int64_t)c * b.count * kBins, x1 = x0 + (int64_t)b.count * kBins;
    const int32_t lo = x0 < nk ? b.nb_off[x0] : (int32_t)carry;
    const int32_t hi = x1 < nk ? b.nb_off[x1] : (int32_t)carry;
    (&b.ctr->num_split_items)[c] = hi - lo;  // split, block, wave, light: consecutive fields
  }
}

__global__ void k_b_num_bin_fill(BatchDev b) {
  __shared__ int32_t cnt[kNumClasses * kBins], base[kNumClasses * kBins];
  __shared__ int32_t nsplit, split_base;
  for (int x = threadIdx.x; x < kNumClasses * kBins; x += blockDim.x) cnt[x] = 0;
  if (threadIdx.x == 0) nsplit = 0;
  __syncthreads();
  const int t = find_inst(b.sb_off, b.count, blockIdx.x);
  const BInst& in = b.insts[t];
  const int64_t r0 = (blockIdx.x - b.sb_off[t]) * (int64_t)kScanRows;
  const int64_t r1 = min((int64_t)in.pr.n, r0 + kScanRows);
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {  // counts of this workgroup's rows
    const int64_t f = in.pr.flops[i];
    if (f > 0) {
      int cls, key, count, ce;
      num_key(f, in.pr.arp[i + 1] - in.pr.arp[i], in.th, cls, key, count, ce);
      atomicAdd(&cnt[key], count);
      if (cls == 0) atomicAdd(&nsplit, 1);
    }
  }
  __syncthreads();
  for (int x = threadIdx.x; x < kNumClasses * kBins; x += blockDim.x) {
    if (cnt[x]) {
      const int k = nb_key(b, x / kBins, in.rank, x % kBins);
      base[x] = b.nb_off[k] + atomicAdd(&b.nb_cur[k], cnt[x]);
    }
    cnt[x] = 0;
  }
  if (threadIdx.x == 0) {
    if (nsplit) split_base = atomicAdd(&b.ctr->num_split_rows, nsplit);
    nsplit = 0;
  }
  __syncthreads();
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const int64_t f = in.pr.flops[i];
    if (f <= 0) continue;
    const int a = in.pr.arp[i], m = in.pr.arp[i + 1] - a;
    int cls, key, count, ce;
    num_key(f, m, in.th, cls, key, count, ce);
    const int pos = base[key] + atomicAdd(&cnt[key], count);
    if (cls == 0) {
      for (int c = 0; c < count; ++c) {
        const int p0 = a + c * ce;
        b.num_items[pos + c] = Item{(int32_t)i, p0, min(a + m, p0 + ce), pos + c};
        b.num_inst[pos + c] = t;
      }
      b.split_rows[split_base + atomicAdd(&nsplit, 1)] = SplitRow{(int32_t)i, pos, count, t};
    } else {
      b.num_items[pos] = Item{(int32_t)i, a, a + m, cls == 1 ? kNoSlot : 0};
      b.num_inst[pos] = t;
    }
  }
}

// ---------------------------------------------------------------- numeric

// One launch per launch class: a workgroup per workgroup item (split
// chunks, then whole rows), then a workgroup per kWavesPerBlock wavefront
// rows. The grid is sized from the counts of the plan's symbolic pass (the
// patterns are fixed); the grid stride only covers larger counts.
template <int GL, int LAYOUT, typename IdxT>
__global__ __launch_bounds__(kBlock) void k_b_numeric(BatchDev b) {
  using S = SemiringT<float>;
  extern __shared__ __align__(16) unsigned char smem[];
  double* strips = (double*)smem;
  int4* stage = (int4*)(smem + (size_t)kWavesPerBlock * b.lds_d * sizeof(double));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int2 r0 = nb_range(b, 0), r1 = nb_range(b, 1), r2 = nb_range(b, 2);
  const int n0 = r0.y - r0.x, n_wg = n0 + (r1.y - r1.x);
  const int n_blocks = n_wg + (r2.y - r2.x + kWavesPerBlock - 1) / kWavesPerBlock;
  for (int g = blockIdx.x; g < n_blocks; g += gridDim.x) {
    if (g < n_wg) {
      const int x = g < n0 ? r0.x + g : r1.x + (g - n0);
      const Item it = b.num_items[x];
      const Problem& pr = b.insts[b.num_inst[x]].pr;
      const int d = pr.d;
      for (int j = threadIdx.x; j < kWavesPerBlock * d; j += kBlock) strips[j] = 0.0;
      __syncthreads();
      accumulate_range<GL, float, BSep<IdxT>, LAYOUT>(pr, it.p0, it.p1, wave, kWavesPerBlock, strips + wave * d,
                                                       stage + wave * kWave);
      __syncthreads();
      for (int j = threadIdx.x; j < d; j += kBlock)
        strips[j] = S::add(S::add(S::add(strips[j], strips[d + j]), strips[2 * d + j]), strips[3 * d + j]);
      __syncthreads();
      if (it.aux != kNoSlot) {
        double* dst = b.partial + (int64_t)it.aux * b.dmax;
        for (int j = threadIdx.x; j < d; j += kBlock) dst[j] = strips[j];
      } else {
        emit_row<float>(pr, it.row, strips, wave, kWavesPerBlock);
      }
      __syncthreads();  // the strips are reused by the next item
    } else {
      const int64_t x = r2.x + (int64_t)(g - n_wg) * kWavesPerBlock + wave;
      if (x < r2.y) {
        const Item it = b.num_items[x];
        const Problem& pr = b.insts[b.num_inst[x]].pr;
        double* strip = strips + wave * b.lds_d;
        for (int j = lane; j < pr.d; j += kWave) strip[j] = 0.0;
        wave_sync();
        accumulate_range<GL, float, BSep<IdxT>, LAYOUT>(pr, it.p0, it.p1, 0, 1, strip, stage + wave * kWave);
        wave_sync();
        emit_row<float>(pr, it.row, strip, 0, 1);
      }
      __syncthreads();  // a later wavefront-row block of this workgroup reuses the strips
    }
  }
}

template <int GL, int LAYOUT, typename IdxT>
__global__ __launch_bounds__(kBlock) void k_b_numeric_light(BatchDev b) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int G = kBlock / GL;
  const int grp = threadIdx.x / GL, gl = threadIdx.x % GL;
  double* strip = (double*)smem + grp * b.lds_d;
  int4* stage = (int4*)(smem + (size_t)G * b.lds_d * sizeof(double)) + grp * GL;
  const int2 r3 = nb_range(b, 3);
  for (int64_t x = r3.x + (int64_t)blockIdx.x * G + grp; x < r3.y; x += (int64_t)gridDim.x * G) {
    const Item it = b.num_items[x];
    const Problem& pr = b.insts[b.num_inst[x]].pr;
    for (int j = gl; j < pr.d; j += GL) strip[j] = 0.0;
    wave_sync();
    accumulate_light<GL, float, BSep<IdxT>, LAYOUT>(pr, it.p0, it.p1, strip, stage, gl);
    wave_sync();
    emit_group<GL, float>(pr, it.row, strip, gl);
    wave_sync();
  }
}

__global__ __launch_bounds__(kBlock) void k_b_split_finalize(BatchDev b) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* strip = (double*)smem;
  const int nrows = b.ctr->num_split_rows;
  for (int r = blockIdx.x; r < nrows; r += gridDim.x) {
    const SplitRow s = b.split_rows[r];
    const Problem& pr = b.insts[s.pad].pr;
    for (int j = threadIdx.x; j < pr.d; j += kBlock) {
      double acc = 0.0;
      for (int c = 0; c < s.count; ++c) acc += b.partial[(int64_t)(s.first + c) * b.dmax + j];
      strip[j] = acc;
    }
    __syncthreads();
    emit_row<float>(pr, s.row, strip, threadIdx.x >> 6, kWavesPerBlock);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- host side

struct Batch {
  int32_t count = 0, dmax = 1, idb = 1;
  // Numeric launch classes: instances with the same group widths, product
  // layout and LDS strip size class run in one pair of launches (heavy and
  // light), their ranks [r_lo, r_hi) adjacent in the work list.
  struct LaunchClass {
    int gl, lgl, flat, dcls, lds_d, r_lo, r_hi;
    int64_t heavy_blocks, light_blocks;  // grids, from the plan's counts
  };
  std::vector<LaunchClass> classes;
  // Symbolic launch groups: instances of one bitmap width, ranks [r_lo, r_hi)
  struct SymGroup {
    int wp, r_lo, r_hi;
    int64_t rows;
  };
  std::vector<SymGroup> sym_groups;
  std::vector<BInst> host_insts;
  DevBuf ebnd;  // per A entry of every instance, its B row bounds (int2), from the plan
  DevBuf insts, offs, work, sym_items, sym_inst, num_items, num_inst, split_rows, partial, block_sums, inst_flops,
      ctr, tmp_rowptrs, tmp_off, nbins;
  int64_t total_rows = 0, total_bm = 0, total_sb = 0, rowptr_total = 0;
  int64_t sym_cap = 0, num_cap = 0, pool = 0;
  BatchDev dev{};
  Counters* host_ctr = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~Batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (host_ctr) (void)hipHostFree(host_ctr);
  }
};

static int enqueue_run(Batch* bt, hipStream_t st, bool numeric) {
  BatchDev b = bt->dev;
  k_b_zero<<<1, 256, 0, st>>>(b.ctr);
  if (bt->total_bm > 0)
    k_b_bitmap<<<(unsigned)bt->total_bm, 256, (size_t)(kBmRows + 1 + kBmRows * bitmap_words(bt->dmax)) * 4, st>>>(b);
  {
    // numeric and symbolic counts and cursors
    int rc = launch_zero_bytes(b.nb_cnt, (size_t)2 * kNumClasses * bt->count * kBins * 4, st);
    if (!rc) rc = launch_zero_bytes(b.sb_cnt, (size_t)2 * bt->count * kBins * 4, st);
    if (rc) return rc;
  }
  if (bt->total_sb > 0) k_b_sym_bin_count<<<(unsigned)bt->total_sb, 256, 0, st>>>(b);
  k_b_sym_bin_scan<<<1, kScanThreads, 0, st>>>(b);
  if (bt->total_sb > 0) k_b_sym_bin_fill<<<(unsigned)bt->total_sb, 256, 0, st>>>(b);
  if (bt->sym_cap > 0) k_b_sym_split_zero<<<grid_for(bt->sym_cap, 256), 256, 0, st>>>(b);
  // one pair of symbolic launches per bitmap width
  for (const auto& g : bt->sym_groups) {
    BatchDev bb = b;
    bb.r_lo = g.r_lo;
    bb.r_hi = g.r_hi;
    if (g.rows == 0) continue;
    const unsigned gl = grid_for(g.rows, kBlock);
    switch (g.wp) {
#define TSS_BSYM(W)                                                  \
  case W:                                                            \
    k_b_sym_light_lanes<W><<<gl, kBlock, 0, st>>>(bb);               \
    k_b_symbolic_lanes<W><<<2048, kBlock, 0, st>>>(bb);              \
    break;
      TSS_BSYM(1) TSS_BSYM(2) TSS_BSYM(4) TSS_BSYM(8)
#undef TSS_BSYM
      default:
        k_b_sym_light<<<grid_for(g.rows, (int64_t)(kWave / g.wp) * kWavesPerBlock), kBlock, 0, st>>>(bb, g.wp);
        k_b_symbolic<<<2048, kBlock, 0, st>>>(bb, g.wp);
    }
  }
  if (bt->total_sb > 0) k_b_count_rows<<<(unsigned)bt->total_sb, kScanThreads, 0, st>>>(b);
  k_b_scan<<<1, kScanThreads, 0, st>>>(b);
  if (bt->total_sb > 0) k_b_write_rowptr<<<(unsigned)bt->total_sb, kScanThreads, 0, st>>>(b);
  k_b_empty_rowptr<<<grid_for(bt->count, 256), 256, 0, st>>>(b);
  if (bt->total_sb > 0) k_b_num_bin_count<<<(unsigned)bt->total_sb, 256, 0, st>>>(b);
  k_b_num_bin_scan<<<1, kScanThreads, 0, st>>>(b);
  if (bt->total_sb > 0) k_b_num_bin_fill<<<(unsigned)bt->total_sb, 256, 0, st>>>(b);
  TSS_CHECK_LAUNCH();
  if (!numeric) return TSSPGEMM_OK;
  // one pair of launches per launch class, each taking the class's ranges
  // of the binned list
#define TSS_BK(K, GLV, L)                                                                              \
  (bt->idb == 1 ? K<GLV, L, uint8_t> : K<GLV, L, uint16_t>)<<<grid, kBlock, lds, st>>>(bb);
#define TSS_BN(GLV)                                                                                    \
  case GLV:                                                                                            \
    if (c.flat == kLayoutFlat)                                                                         \
      TSS_BK(k_b_numeric, GLV, kLayoutFlat)                                                            \
    else if (c.flat == kLayoutVec)                                                                     \
      TSS_BK(k_b_numeric, GLV, kLayoutVec)                                                             \
    else                                                                                               \
      TSS_BK(k_b_numeric, GLV, kLayoutRows)                                                            \
    break;
#define TSS_BL(GLV)                                                                                    \
  case GLV:                                                                                            \
    if (c.flat == kLayoutFlat)                                                                         \
      TSS_BK(k_b_numeric_light, GLV, kLayoutFlat)                                                      \
    else if (c.flat == kLayoutVec)                                                                     \
      TSS_BK(k_b_numeric_light, GLV, kLayoutVec)                                                       \
    else                                                                                               \
      TSS_BK(k_b_numeric_light, GLV, kLayoutRows)                                                      \
    break;
  for (size_t ci = 0; ci < bt->classes.size(); ++ci) {
    const Batch::LaunchClass& c = bt->classes[ci];
    BatchDev bb = b;
    bb.r_lo = c.r_lo;
    bb.r_hi = c.r_hi;
    bb.lds_d = c.lds_d;
    if (c.heavy_blocks > 0) {
      const unsigned grid = (unsigned)c.heavy_blocks;
      const size_t lds = (size_t)kWavesPerBlock * c.lds_d * 8 + kWavesPerBlock * kWave * sizeof(int4);
      switch (c.gl) {
        TSS_BN(4) TSS_BN(8) TSS_BN(16) TSS_BN(32) TSS_BN(64)
        default: set_error("batched: bad group width"); return TSSPGEMM_ERR_INVALID_ARG;
      }
    }
    if (c.light_blocks > 0) {
      const unsigned grid = (unsigned)c.light_blocks;
      const size_t lds = (size_t)(kBlock / c.lgl) * c.lds_d * 8 + kBlock * sizeof(int4);
      switch (c.lgl) {
        TSS_BL(4) TSS_BL(8) TSS_BL(16) TSS_BL(32) TSS_BL(64)
        default: set_error("batched: bad light group width"); return TSSPGEMM_ERR_INVALID_ARG;
      }
    }
  }
#undef TSS_BN
#undef TSS_BL
#undef TSS_BK
  TSS_CHECK_LAUNCH();
  k_b_split_finalize<<<1024, kBlock, (size_t)bt->dmax * 8, st>>>(b);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

int light_group_lanes(int group_lanes, int64_t d, int sr);

static int batch_plan(int32_t count, const tsspgemm_csr* As, const tsspgemm_csr* Bs, const tsspgemm_tuning* tunes,
                      Batch* bt, int64_t* pool_capacity, int64_t* rowptr_total, hipStream_t st) {
  int rc;
  if (count < 0 || (count > 0 && (!As || !Bs)) || !pool_capacity || !rowptr_total) {
    set_error("batched_plan: bad arguments");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  bt->count = count;
  std::vector<int64_t> row_off(count + 1, 0), bm_off(count + 1, 0), sb_off(count + 1, 0);
  int64_t ws_bytes = 0, sym_cap = 0, num_cap = 0, rp_total = 0;
  std::vector<int64_t> ws_at(count);
  int dmax = 1;
  for (int t = 0; t < count; ++t) {
    const tsspgemm_csr *A = &As[t], *B = &Bs[t];
    if ((rc = check_csr(A, "A", true)) || (rc = check_csr(B, "B", true))) {
      set_error("batched_plan: instance " + std::to_string(t) + ": " + get_error());
      return rc;
    }
    if (A->nrows != A->ncols || B->nrows != A->ncols) {
      set_error("batched_plan: instance " + std::to_string(t) + ": A must be n x n and B n x d");
      return TSSPGEMM_ERR_INVALID_ARG;
    }
    if (B->ncols > kMaxDenseD) {
      set_error("batched_plan: instance " + std::to_string(t) + ": d > 1024");
      return TSSPGEMM_ERR_UNSUPPORTED;
    }
    const int64_t n = A->nrows;
    const int wp = bitmap_words(B->ncols);
    dmax = std::max<int>(dmax, (int)B->ncols);
    row_off[t + 1] = row_off[t] + n;
    bm_off[t + 1] = bm_off[t] + (n + kBmRows - 1) / kBmRows;
    sb_off[t + 1] = sb_off[t] + (n + kScanRows - 1) / kScanRows;
    ws_at[t] = ws_bytes;
    ws_bytes += ((2 * n * wp * 4 + n * 8 + n * 4) + 255) / 256 * 256;
    ws_bytes += (B->nnz * 2 + 255) / 256 * 256;  // narrowed column ids (at most 2 bytes each)
    rp_total += n + 1;
    num_cap += 2 * n + A->nnz / 64 + 2;
  }
  bt->dmax = dmax;
  bt->idb = dmax <= 256 ? 1 : 2;
  // Without tunings the batch runs one group width and product layout, from
  // the mean B row length over all instances (one launch per phase; measured
  // faster on mixed batches than each instance's own default). With tunings,
  // each instance keeps its own.
  int batch_gl = 0, batch_products = TSSPGEMM_PRODUCTS_AUTO;
  {
    int64_t bn = 0, bnnz = 0;
    for (int t = 0; t < count; ++t) {
      bn += Bs[t].nrows;
      bnnz += Bs[t].nnz;
    }
    const tsspgemm_csr mean_b{bn, dmax, bnnz, nullptr, nullptr, nullptr};
    tsspgemm_tuning t0;
    resolve_tuning(tunes ? &tunes[0] : nullptr, &mean_b, &t0);
    // 4096 measured slower than 2048 on the 64-instance batch, whose rows are
    // short (6.26 against 6.22 ms)
    bt->dev.sym_split = tunes && tunes[0].sym_split_nnz > 0 ? tunes[0].sym_split_nnz : kBatchSymSplit;
    batch_gl = t0.group_lanes;
    batch_products = t0.products;
  }
  // symbolic items: one per heavy row, one per chunk of the batch's split
  // size (the first tuning's, for every instance)
  for (int t = 0; t < count; ++t) sym_cap += As[t].nrows + As[t].nnz / bt->dev.sym_split + 2;
  bt->total_rows = row_off[count];
  bt->total_bm = bm_off[count];
  bt->total_sb = sb_off[count];
  bt->rowptr_total = rp_total;
  bt->sym_cap = sym_cap;
  bt->num_cap = num_cap;
  if ((rc = bt->insts.ensure(sizeof(BInst) * (count + 1))) || (rc = bt->offs.ensure(sizeof(int64_t) * 5 * (count + 1))) ||
      (rc = bt->work.ensure((size_t)ws_bytes + 256)) || (rc = bt->sym_items.ensure(sizeof(Item) * (sym_cap + 1))) ||
      (rc = bt->sym_inst.ensure(4 * (sym_cap + 1))) || (rc = bt->num_items.ensure(sizeof(Item) * (num_cap + 1))) ||
      (rc = bt->num_inst.ensure(4 * (num_cap + 1))) ||
      (rc = bt->split_rows.ensure(sizeof(SplitRow) * (bt->total_rows + 1))) ||
      (rc = bt->block_sums.ensure(16 * (bt->total_sb + 1))) || (rc = bt->inst_flops.ensure(8 * (count + 1))) ||
      (rc = bt->ctr.ensure(sizeof(Counters))) || (rc = bt->tmp_rowptrs.ensure(4 * (rp_total + 1))) ||
      (rc = bt->nbins.ensure((size_t)3 * (kNumClasses + 1) * (count + 1) * kBins * 4)) ||
      (rc = bt->tmp_off.ensure(8 * (count + 1))))
    return rc;
  int64_t a_nnz_total = 0;
  for (int t = 0; t < count; ++t) a_nnz_total += As[t].nnz;
  if ((rc = bt->ebnd.ensure(sizeof(int2) * (a_nnz_total + 1)))) return rc;
  TSS_HIP(hipHostMalloc((void**)&bt->host_ctr, sizeof(Counters), hipHostMallocDefault));
  bt->host_insts.resize(count);
  int64_t a_off = 0;
  int64_t rp_off = 0;
  std::vector<int64_t> rank_t(count + 1, 0), rrow_off(count + 1, 0);
  for (int t = 0; t < count; ++t) {
    const tsspgemm_csr *A = &As[t], *B = &Bs[t];
    const int64_t n = A->nrows;
    const int wp = bitmap_words(B->ncols);
    char* base = (char*)bt->work.p + ws_at[t];
    BInst& in = bt->host_insts[t];
    in = BInst{};
    in.pr.n = (int32_t)n;
    in.pr.d = (int32_t)B->ncols;
    in.pr.wp = wp;
    in.pr.arp = A->rowptr;
    in.pr.aci = A->colidx;
    in.pr.aval = A->vals;
    in.pr.brp = B->rowptr;
    in.pr.bci = B->colidx;
    in.pr.bval = B->vals;
    in.pr.bbits = (const uint32_t*)base;
    in.pr.cbits = (uint32_t*)(base + n * wp * 4);
    in.pr.flops = (int64_t*)(base + 2 * n * wp * 4);
    in.cnt = (int32_t*)(base + 2 * n * wp * 4 + n * 8);
    in.pr.bcol = base + ((2 * n * wp * 4 + n * 8 + n * 4) + 255) / 256 * 256;
    int2* eb = (int2*)bt->ebnd.p + a_off;
    in.pr.ebnd = eb;
    if (A->nnz > 0) {
      const unsigned g = (unsigned)std::min<int64_t>((A->nnz + 255) / 256, 8192);
      k_b_entry_bounds<<<g, 256, 0, st>>>(A->colidx, B->rowptr, A->nnz, eb);
      TSS_CHECK_LAUNCH();
    }
    a_off += A->nnz;
    tsspgemm_tuning tn;
    resolve_tuning(tunes ? &tunes[t] : nullptr, B, &tn);
    if (!tunes) {
      tn.group_lanes = batch_gl;
      tn.products = batch_products;
    }
    in.th = NumThresholds{tn.light_max_flops, tn.wave_max_flops, tn.split_flops};
    in.rp_off = rp_off;
    // the instance's group width and product layout (its own tuning's, or the
    // batch's when no tunings are given)
    in.flat = tn.products == TSSPGEMM_PRODUCTS_FLAT ? kLayoutFlat
              : (tn.products == TSSPGEMM_PRODUCTS_VEC4 && ((uintptr_t)B->vals % 16) == 0 ? kLayoutVec : kLayoutRows);
    in.gl = in.flat == kLayoutFlat ? 64 : tn.group_lanes;
    in.lgl = light_group_lanes(tn.group_lanes, B->ncols, TSSPGEMM_PLUS_TIMES_F32);
    rp_off += n + 1;
  }
  // Launch classes: the strip size class is the smallest power of two >= 32
  // holding d, so instances with narrow B get small strips (more resident
  // wavefronts) rather than the batch's widest. Instances are ranked class
  // by class (size class first, so that one bitmap width is one range of
  // ranks), in their order within a class.
  {
    auto dcls = [](int d) {
      int c = 32;
      while (c < d) c <<= 1;
      return c;
    };
    std::vector<int> order(count);
    for (int t = 0; t < count; ++t) order[t] = t;
    auto key = [&](int t) {
      const BInst& in = bt->host_insts[t];
      return std::array<int, 4>{dcls(in.pr.d), in.flat, in.gl, in.lgl};
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key(x) < key(y); });
    bt->classes.clear();
    bt->sym_groups.clear();
    for (int r = 0; r < count; ++r) {
      const int t = order[r];
      BInst& in = bt->host_insts[t];
      in.rank = r;
      const auto k = key(t);
      if (bt->classes.empty() || bt->classes.back().dcls != k[0] || bt->classes.back().flat != k[1] ||
          bt->classes.back().gl != k[2] || bt->classes.back().lgl != k[3])
        bt->classes.push_back({k[2], k[3], k[1], k[0], 1, r, r, 0, 0});
      Batch::LaunchClass& c = bt->classes.back();
      c.r_hi = r + 1;
      c.lds_d = std::max(c.lds_d, (int)in.pr.d);
      if (bt->sym_groups.empty() || bt->sym_groups.back().wp != in.pr.wp)
        bt->sym_groups.push_back({in.pr.wp, r, r, 0});
      bt->sym_groups.back().r_hi = r + 1;
      bt->sym_groups.back().rows += in.pr.n;
      rank_t[r] = t;
      rrow_off[r + 1] = rrow_off[r] + in.pr.n;
    }
  }
  int64_t* offs = (int64_t*)bt->offs.p;
  TSS_HIP(hipMemcpyAsync(bt->insts.p, bt->host_insts.data(), sizeof(BInst) * count, hipMemcpyHostToDevice, st));
  TSS_HIP(hipMemcpyAsync(offs, row_off.data(), 8 * (count + 1), hipMemcpyHostToDevice, st));
  TSS_HIP(hipMemcpyAsync(offs + (count + 1), bm_off.data(), 8 * (count + 1), hipMemcpyHostToDevice, st));
  TSS_HIP(hipMemcpyAsync(offs + 2 * (count + 1), rrow_off.data(), 8 * (count + 1), hipMemcpyHostToDevice, st));
  TSS_HIP(hipMemcpyAsync(offs + 4 * (count + 1), rank_t.data(), 8 * (count + 1), hipMemcpyHostToDevice, st));
  TSS_HIP(hipMemcpyAsync(offs + 3 * (count + 1), sb_off.data(), 8 * (count + 1), hipMemcpyHostToDevice, st));
  BatchDev& b = bt->dev;
  b.insts = (BInst*)bt->insts.p;
  b.count = count;
  b.dmax = dmax;
  b.idb = bt->idb;
  b.row_off = offs;
  b.bm_off = offs + (count + 1);
  b.rrow_off = offs + 2 * (count + 1);
  b.rank_t = offs + 4 * (count + 1);
  b.sb_off = offs + 3 * (count + 1);
  b.total_rows = bt->total_rows;
  b.total_sb = bt->total_sb;
  b.sym_items = (Item*)bt->sym_items.p;
  b.sym_inst = (int32_t*)bt->sym_inst.p;
  b.num_items = (Item*)bt->num_items.p;
  b.num_inst = (int32_t*)bt->num_inst.p;
  b.split_rows = (SplitRow*)bt->split_rows.p;
  b.block_sums = (int64_t*)bt->block_sums.p;
  b.inst_flops = (int64_t*)bt->inst_flops.p;
  b.nb_cnt = (int32_t*)bt->nbins.p;
  b.nb_cur = b.nb_cnt + (size_t)kNumClasses * count * kBins;
  b.nb_off = b.nb_cur + (size_t)kNumClasses * count * kBins;
  b.sb_cnt = b.nb_off + (size_t)kNumClasses * count * kBins + kBins;
  b.sb_cur = b.sb_cnt + (size_t)count * kBins;
  b.sb_kof = b.sb_cur + (size_t)count * kBins;
  b.ctr = (Counters*)bt->ctr.p;
  // a symbolic pass at plan time sizes the output pool and the split slots
  b.c_rowptrs = (int32_t*)bt->tmp_rowptrs.p;
  b.pool_ci = nullptr;
  b.pool_val = nullptr;
  b.c_off = (int64_t*)bt->tmp_off.p;
  b.partial = nullptr;
  if ((rc = enqueue_run(bt, st, false))) return rc;
  TSS_HIP(hipMemcpyAsync(bt->host_ctr, b.ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  const size_t nk = (size_t)kNumClasses * count * kBins;
  std::vector<int32_t> koff(nk + 1);
  TSS_HIP(hipMemcpyAsync(koff.data(), b.nb_off, (nk + 1) * 4, hipMemcpyDeviceToHost, st));
  TSS_HIP(hipStreamSynchronize(st));
  bt->pool = bt->host_ctr->nnz_total;
  // grids of the numeric launches: the work list's counts per launch class
  // (fixed, since the patterns are)
  for (auto& c : bt->classes) {
    auto range = [&](int cls) {
      return (int64_t)koff[((size_t)cls * count + c.r_hi) * kBins] - koff[((size_t)cls * count + c.r_lo) * kBins];
    };
    c.heavy_blocks = range(0) + range(1) + (range(2) + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t per_block = kBlock / c.lgl;
    // one workgroup per kBlock / lgl light rows (capped at 2048 grid-striding
    // workgroups the replay took 6.22 ms instead of 6.14)
    c.light_blocks = std::min<int64_t>((range(3) + per_block - 1) / per_block, 1 << 20);
    c.heavy_blocks = std::min<int64_t>(c.heavy_blocks, INT32_MAX);
  }
  if ((rc = bt->partial.ensure((size_t)(bt->host_ctr->num_split_items + 1) * dmax * 8))) return rc;
  b.partial = (double*)bt->partial.p;
  *pool_capacity = bt->pool;
  *rowptr_total = rp_total;
  return TSSPGEMM_OK;
}

static int batch_bind(Batch* bt, int32_t* c_rowptrs, int32_t* pool_colidx, float* pool_vals, int64_t* c_offsets) {
  if (!bt || !c_rowptrs || !c_offsets || (bt->pool > 0 && (!pool_colidx || !pool_vals))) {
    set_error("batched_run: NULL argument");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  bt->dev.c_rowptrs = c_rowptrs;
  bt->dev.pool_ci = pool_colidx;
  bt->dev.pool_val = pool_vals;
  bt->dev.c_off = c_offsets;
  return TSSPGEMM_OK;
}

}  // namespace tss

using namespace tss;

extern "C" {

int tsspgemm_batched_plan(int32_t count, const tsspgemm_csr* As, const tsspgemm_csr* Bs, const tsspgemm_tuning* tune,
                          tsspgemm_batch* out, int64_t* pool_capacity, int64_t* rowptr_total, void* stream) {
  try {
    if (!out) {
      set_error("batched_plan: out is NULL");
      return TSSPGEMM_ERR_INVALID_ARG;
    }
    Batch* bt = new (std::nothrow) Batch();
    if (!bt) {
      set_error("out of host memory");
      return TSSPGEMM_ERR_NOMEM;
    }
    int rc = batch_plan(count, As, Bs, tune, bt, pool_capacity, rowptr_total, (hipStream_t)stream);
    if (rc) {
      delete bt;
      *out = nullptr;
      return rc;
    }
    *out = (tsspgemm_batch)bt;
    return TSSPGEMM_OK;
  } catch (...) {
    set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}

int tsspgemm_batched_run(tsspgemm_batch batch, int32_t* c_rowptrs, int32_t* pool_colidx, float* pool_vals,
                         int64_t* c_offsets, void* stream) {
  Batch* bt = (Batch*)batch;
  int rc = batch_bind(bt, c_rowptrs, pool_colidx, pool_vals, c_offsets);
  if (rc) return rc;
  return enqueue_run(bt, (hipStream_t)stream, true);
}

int tsspgemm_batched_capture(tsspgemm_batch batch, int32_t* c_rowptrs, int32_t* pool_colidx, float* pool_vals,
                             int64_t* c_offsets) {
  Batch* bt = (Batch*)batch;
  int rc = batch_bind(bt, c_rowptrs, pool_colidx, pool_vals, c_offsets);
  if (rc) return rc;
  if (bt->exec) {
    (void)hipGraphExecDestroy(bt->exec);
    bt->exec = nullptr;
  }
  if (bt->graph) {
    (void)hipGraphDestroy(bt->graph);
    bt->graph = nullptr;
  }
  if (!bt->cap_stream) TSS_HIP(hipStreamCreateWithFlags(&bt->cap_stream, hipStreamNonBlocking));
  TSS_HIP(hipStreamBeginCapture(bt->cap_stream, hipStreamCaptureModeThreadLocal));
  rc = enqueue_run(bt, bt->cap_stream, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(bt->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    return TSSPGEMM_ERR_HIP;
  }
  bt->graph = g;
  TSS_HIP(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
  return TSSPGEMM_OK;
}

int tsspgemm_batched_launch(tsspgemm_batch batch, void* stream) {
  Batch* bt = (Batch*)batch;
  if (!bt || !bt->exec) {
    set_error("batched_launch: no captured graph (call tsspgemm_batched_capture first)");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  TSS_HIP(hipGraphLaunch(bt->exec, (hipStream_t)stream));
  return TSSPGEMM_OK;
}

int tsspgemm_batched_flops(tsspgemm_batch batch, int64_t* flops_host) {
  Batch* bt = (Batch*)batch;
  if (!bt || !flops_host) {
    set_error("batched_flops: NULL argument");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (bt->count > 0)
    TSS_HIP(hipMemcpy(flops_host, bt->inst_flops.p, 8 * bt->count, hipMemcpyDeviceToHost));
  return TSSPGEMM_OK;
}

void tsspgemm_batched_destroy(tsspgemm_batch batch) { delete (Batch*)batch; }

}  // extern "C"
