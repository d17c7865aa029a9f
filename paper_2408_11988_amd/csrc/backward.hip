// Backward of C = A B for a loss L with G = dL/dC given on C's pattern.
//
//  dL/dA(i,k) = sum over j in pat(B_k) of G(i,j) B(k,j)   (an SDDMM on pat(A))
//  dL/dB(k,j) = sum over i in pat(A^T_k) of A(i,k) G(i,j) (A^T G sampled on pat(B))
//
// Every needed G(i,j) lies in pat(C): if A(i,k) and B(k,j) are stored, the
// structural product stores C(i,j). Both gradients accumulate in FP64 in a
// fixed order and round once to FP32.
//
// First pass, over A's rows (the forward plan's binned rows): a row's G
// values are staged in an LDS strip of width d; each A entry (i,k) is a dot
// product of B row k with that strip (dL/dA), taken by a group of GL lanes
// and reduced across the group. For dL/dB the same walk copies A(i,k) and
// every G(i,j) it reads (FP32 values, not rounded) into a block per A entry:
// A(i,k), then G(i, pat(B_k)) in B row order, zero-padded to a slot of a
// multiple of 16 floats (64 bytes). Slots are placed in A^T order, so the
// group's lanes write whole 64-byte segments at scattered places.
//
// Second pass, over A^T (from tsspgemm_transpose): B row k's blocks are one
// contiguous range. A group of GL lanes takes the slot positions of B row k
// (lane = entry) and runs over the entries i of A^T row k in order, adding
// A(i,k) G(i,j). Long A^T rows are cut into chunks whose partial sums a
// third kernel adds in chunk order.
//
// Measured at R-MAT 20 x 256 (5%), per call: a single pass over A^T that
// looked G(i,j) up in C's row i (a record of C's bitmap word plus a
// popcount) fetched about 15 GB; blocks without A(i,k), read with A(i,k)
// gathered through the permutation, 11.6 GB in the second pass (a cache
// line per pair for the gather alone); blocks packed back to back in A
// order made the first pass's writes contiguous but the second pass a
// gather of one or two cache lines per pair; packed blocks in A^T order
// scattered the first pass's writes in 32- and 64-byte pieces. The padded
// A^T-order slots keep the second pass one contiguous read (about 3.4 GB,
// 0.8 ms) with whole-segment writes in the first.
#include "api_internal.hpp"
#include "dev_numeric.hpp"

namespace tss {

constexpr int kGbChunk = 512;  // A^T entries per dL/dB work item

__device__ __forceinline__ void gsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the GL lanes of a group (lanes aligned to GL), FP64.
template <int GL>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = 1; o < GL; o <<= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

struct GradAParams {
  Problem pr;             // A, B, C pattern (crp, cbits) of the forward plan
  const int32_t* gci;     // G = dL/dC on C's pattern
  const float* gval;
  float* grad_a;          // dL/dA, or null (only the sampled G is written)
  float* gbuf;            // sampled G for dL/dB, or null: per A entry (i,k) a block of A(i,k) then G(i, pat(B_k))
  const int32_t* slot_a;  // per A entry: start of its block in gbuf in 16-float units (-1: its B row is empty)
  const Item* items;
  int32_t n_wg_items, n_heavy_records, n_light;
};

// Floats of the slot of a block of a B row of len entries: A(i,k) and the
// len G values, rounded up to 16 floats (64 bytes); none for an empty row.
__device__ __forceinline__ int gb_slot(int len) { return len > 0 ? 16 * ((len + 16) / 16) : 0; }

// Dot products of staged A entries: stage[e] = (start, end) of B row k for
// the entry base + e of the row, e in [0, nb); group grp of ngroups takes
// blocks of U entries grp * U, (grp + ngroups) * U, ... Lanes of a group walk
// the B row (column ids narrowed to IdxT) against the row's G strip; each dot
// product is summed over the group in FP64 and rounded once.
//
// With GATHER the stage also holds the entry's slot in gbuf (in 16-float
// units) and A(i,k), and lane gl walks the slot's positions gl, gl + GL, ...
// instead of the B row's entries: position 0 takes A(i,k), position p >= 1
// takes G(i, j) for the (p-1)-th entry (k, j) of B row k (the same product
// the dot product uses), and positions past the row's end take 0. The lanes
// of a group thus write whole 64-byte segments, with no partial writes.
template <int GL, typename IdxT, bool GATHER>
__device__ __forceinline__ void grad_a_staged(const GradAParams& gp, int base, int nb, const int4* stage, int grp,
                                              int ngroups, const float* strip) {
  constexpr int U = 4;
  const int gl = threadIdx.x % GL;
  const Problem& pr = gp.pr;
  const float* __restrict__ bval = (const float*)pr.bval;
  const IdxT* __restrict__ bci = col_ids<IdxT>(pr);
  float* __restrict__ gbuf = gp.gbuf;
  for (int e0 = grp * U; e0 < nb; e0 += ngroups * U) {
    int q0[U], qe[U];
    int64_t w[U];  // GATHER: start of the slot
    float av[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int4 r = make_int4(0, 0, -1, 0);
      if (e0 + u < nb) r = stage[e0 + u];
      q0[u] = r.x;
      qe[u] = r.y;
      w[u] = 16 * (int64_t)r.z;
      av[u] = __builtin_bit_cast(float, r.w);
    }
    // the first GL positions (GATHER) or entries of each row
    const int sh = GATHER ? 1 : 0;  // position p holds entry p - 1
    int jj[U];
    float bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0[u] + gl - sh;
      jj[u] = 0;
      bv[u] = 0.0f;
      if (q >= q0[u] && q < qe[u]) {
        jj[u] = bci[q];
        bv[u] = bval[q];
      }
    }
    double sum[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = q0[u] + gl - sh;
      const bool in = q >= q0[u] && q < qe[u];
      const float g = in ? strip[jj[u]] : 0.0f;
      sum[u] = in ? (double)bv[u] * (double)g : 0.0;
      if constexpr (GATHER) {
        const int S = gb_slot(qe[u] - q0[u]);
        if (gl < S) __builtin_nontemporal_store(gl == 0 ? av[u] : g, gbuf + w[u] + gl);
        for (int p = gl + GL; p < S; p += GL) {
          const int t = q0[u] + p - 1;
          float gt = 0.0f;
          if (t < qe[u]) {
            gt = strip[bci[t]];
            sum[u] += (double)bval[t] * (double)gt;
          }
          __builtin_nontemporal_store(gt, gbuf + w[u] + p);
        }
      } else {
        for (int t = q + GL; t < qe[u]; t += GL) sum[u] += (double)bval[t] * (double)strip[bci[t]];
      }
    }
    if (gp.grad_a) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double v = group_sum<GL>(sum[u]);
        if (gl == 0 && e0 + u < nb) gp.grad_a[base + e0 + u] = (float)v;
      }
    }
  }
}

// Stage entries [base, base + nb) of A (nb <= the caller's lanes): lane t of
// the stagers loads entry base + t and its B row bounds, and (GATHER) its
// slot in gbuf (16-float units) and A(i,k).
template <bool GATHER>
__device__ __forceinline__ void grad_a_stage(const GradAParams& gp, int base, int nb, int t, int4* stage) {
  int4 e = make_int4(0, 0, -1, 0);
  if (t < nb) {
    const int2 bnd = entry_bounds(gp.pr, base + t);
    e.x = bnd.x;
    e.y = bnd.y;
    if constexpr (GATHER) {
      e.z = gp.slot_a[base + t];
      e.w = __builtin_bit_cast(int32_t, ((const float*)gp.pr.aval)[base + t]);
    }
  }
  stage[t] = e;
}

// Workgroup items (split chunks, workgroup rows) and wavefront rows. A
// wavefront stages 64 A entries at a time (coalesced) and its 64/GL groups
// share them.
template <int GL, typename IdxT, bool GATHER>
__global__ __launch_bounds__(kBlock) void k_grad_a(GradAParams gp) {
  extern __shared__ __align__(16) float gstrip[];
  const Problem& pr = gp.pr;
  const int d = pr.d;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = blockIdx.x;
  constexpr int GPW = kWave / GL;
  int4* stage = (int4*)(gstrip + kWavesPerBlock * ((d + 3) & ~3)) + wave * kWave;
  if (g < gp.n_wg_items) {
    const Item it = gp.items[g];
    float* strip = gstrip;
    for (int q = pr.crp[it.row] + threadIdx.x; q < pr.crp[it.row + 1]; q += kBlock) strip[gp.gci[q]] = gp.gval[q];
    __syncthreads();
    for (int base = it.p0 + kWave * wave; base < it.p1; base += kWave * kWavesPerBlock) {
      const int nb = min(kWave, it.p1 - base);
      grad_a_stage<GATHER>(gp, base, nb, lane, stage);
      wave_sync();
      grad_a_staged<GL, IdxT, GATHER>(gp, base, nb, stage, lane / GL, GPW, strip);
      wave_sync();
    }
  } else {
    const int64_t idx = (int64_t)gp.n_wg_items + 4 * (int64_t)(g - gp.n_wg_items) + wave;
    if (idx >= gp.n_heavy_records) return;
    const Item it = gp.items[idx];
    float* strip = gstrip + wave * d;
    for (int q = pr.crp[it.row] + lane; q < pr.crp[it.row + 1]; q += kWave) strip[gp.gci[q]] = gp.gval[q];
    wave_sync();
    for (int base = it.p0; base < it.p1; base += kWave) {
      const int nb = min(kWave, it.p1 - base);
      grad_a_stage<GATHER>(gp, base, nb, lane, stage);
      wave_sync();
      grad_a_staged<GL, IdxT, GATHER>(gp, base, nb, stage, lane / GL, GPW, strip);
      wave_sync();
    }
  }
}

// Light rows: one group (one strip, GL staged entries) per row.
template <int GL, typename IdxT, bool GATHER>
__global__ __launch_bounds__(kBlock) void k_grad_a_light(GradAParams gp) {
  extern __shared__ __align__(16) float gstrip[];
  constexpr int G = kBlock / GL;
  const Problem& pr = gp.pr;
  const int grp = threadIdx.x / GL, gl = threadIdx.x % GL;
  float* strip = gstrip + grp * pr.d;
  int4* stage = (int4*)(gstrip + G * ((pr.d + 3) & ~3)) + grp * GL;
  const Item* items = gp.items + gp.n_heavy_records;
  for (int64_t t = (int64_t)blockIdx.x * G + grp; t < gp.n_light; t += (int64_t)gridDim.x * G) {
    const Item it = items[t];
    for (int q = pr.crp[it.row] + gl; q < pr.crp[it.row + 1]; q += GL) strip[gp.gci[q]] = gp.gval[q];
    for (int base = it.p0; base < it.p1; base += GL) {
      const int nb = min(GL, it.p1 - base);
      grad_a_stage<GATHER>(gp, base, nb, gl, stage);
      wave_sync();
      grad_a_staged<GL, IdxT, GATHER>(gp, base, nb, stage, 0, 1, strip);
      wave_sync();
    }
  }
}

// A entries of rows without products (every B row empty) get 0.
__global__ void k_zero_f32(float* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// ---------------------------------------------------------------- dL/dB

struct GradBParams {
  Problem pr;                // A values, B pattern
  const int32_t* atrp;       // A^T row pointers (n + 1)
  float* grad_b;
  const float* gbuf;         // blocks written by the first pass, in A^T order
  const int64_t* off;        // start of B row k's blocks in gbuf
  Item* items;               // [split chunks][whole rows]: row = k, [p0,p1) range of A^T entries
  SplitRow* split_rows;
  double* partial;           // chunk partial sums (slot x d)
  Counters* ctr;             // num_count/num_cursor classes 0 (chunks) and 3 (rows)
};

// cost of B row k: A^T entries x B entries
__global__ void k_gb_bin_count(GradBParams gb) {
  __shared__ int32_t hist[2 * kBins];
  if (threadIdx.x < 2 * kBins) hist[threadIdx.x] = 0;
  __syncthreads();
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < gb.pr.n) {
    const int m = gb.atrp[k + 1] - gb.atrp[k];
    const int lb = gb.pr.brp[k + 1] - gb.pr.brp[k];
    if (m > 0 && lb > 0) {
      if (m > kGbChunk)
        atomicAdd(&hist[0], (m + kGbChunk - 1) / kGbChunk);
      else
        atomicAdd(&hist[kBins + (kBins - 1 - (31 - __clz(m * lb)))], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * kBins && hist[threadIdx.x]) {
    const int cls = threadIdx.x < kBins ? 0 : 3;
    atomicAdd(&gb.ctr->num_count[cls][threadIdx.x % kBins], hist[threadIdx.x]);
  }
}

__global__ void k_gb_bin_scan(Counters* ctr) {
  int32_t off = 0;
  int32_t tot[2] = {0, 0};
  const int cls[2] = {0, 3};
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < kBins; ++b) {
      ctr->num_cursor[cls[c]][b] = off;
      off += ctr->num_count[cls[c]][b];
      tot[c] += ctr->num_count[cls[c]][b];
    }
  ctr->num_split_items = tot[0];
  ctr->num_light_rows = tot[1];
}

__global__ void k_gb_bin_fill(GradBParams gb) {
  __shared__ int32_t cnt[2 * kBins], base[2 * kBins];
  __shared__ int32_t nsplit, split_base;
  if (threadIdx.x < 2 * kBins) cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) nsplit = 0;
  __syncthreads();
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int a = 0, m = 0, key = -1, count = 0, local = 0, slocal = 0;
  if (k < gb.pr.n) {
    a = gb.atrp[k];
    m = gb.atrp[k + 1] - a;
    const int lb = gb.pr.brp[k + 1] - gb.pr.brp[k];
    if (m > 0 && lb > 0) {
      if (m > kGbChunk) {
        key = 0;
        count = (m + kGbChunk - 1) / kGbChunk;
        slocal = atomicAdd(&nsplit, 1);
      } else {
        key = kBins + (kBins - 1 - (31 - __clz(m * lb)));
        count = 1;
      }
      local = atomicAdd(&cnt[key], count);
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * kBins && cnt[threadIdx.x]) {
    const int cls = threadIdx.x < kBins ? 0 : 3;
    base[threadIdx.x] = atomicAdd(&gb.ctr->num_cursor[cls][threadIdx.x % kBins], cnt[threadIdx.x]);
  }
  if (threadIdx.x == 0 && nsplit) split_base = atomicAdd(&gb.ctr->num_split_rows, nsplit);
  __syncthreads();
  if (count == 0) return;
  const int pos = base[key] + local;
  if (key == 0) {
    for (int c = 0; c < count; ++c) {
      const int p0 = a + c * kGbChunk;
      gb.items[pos + c] = Item{(int32_t)k, p0, min(a + m, p0 + kGbChunk), pos + c};
    }
    gb.split_rows[split_base + slocal] = SplitRow{(int32_t)k, pos, count, 0};
  } else {
    gb.items[pos] = Item{(int32_t)k, a, a + m, kNoSlot};
  }
}

// dL/dB from the blocks written by the first pass. Blocks are in A^T order:
// B row k's blocks, one slot of S = gb_slot(nnz(B_k)) floats per entry of
// A^T row k in order, start at off[k], so an item reads one contiguous range.
// A group of GL lanes takes the slot positions in windows of GL (position
// p = window + gl holds G(i, j) of B row k's entry p - 1; position 0 holds
// A(i,k)); a lane's sum runs over the item's A^T entries in order. Each
// block is one load per lane; A(i,k) comes from the group's lane 0 by a
// shuffle in the first window and by a load in later ones. U blocks are
// read before their sums.
template <int GL>
__global__ __launch_bounds__(kBlock) void k_grad_b_blocks(GradBParams gb) {
  constexpr int G = kBlock / GL;
  constexpr int U = 8;
  const int grp = threadIdx.x / GL, gl = threadIdx.x % GL;
  const int lane0 = (threadIdx.x & (kWave - 1)) & ~(GL - 1);  // the group's first lane in the wavefront
  const Problem& pr = gb.pr;
  const float* __restrict__ gbuf = gb.gbuf;
  const int total = gb.ctr->num_split_items + gb.ctr->num_light_rows;
  for (int64_t t = (int64_t)blockIdx.x * G + grp; t < total; t += (int64_t)gridDim.x * G) {
    const Item it = gb.items[t];
    const int k = it.row;
    const int q0 = pr.brp[k], len = pr.brp[k + 1] - q0;
    const int S = gb_slot(len);
    const float* blk = gbuf + gb.off[k] + (int64_t)(it.p0 - gb.atrp[k]) * S;
    const int nx = it.p1 - it.p0;
    for (int pw = 0; pw <= len; pw += GL) {  // windows holding positions 1..len
      const int pos = pw + gl, e = pos - 1;
      const bool own = e >= 0 && e < len;
      const bool load = pos < S;
      double acc = 0.0;
      for (int x0 = 0; x0 < nx; x0 += U) {
        float v[U], a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = (load && x0 + u < nx) ? blk[(int64_t)(x0 + u) * S + pos] : 0.0f;
        if (pw == 0) {
#pragma unroll
          for (int u = 0; u < U; ++u) a[u] = __shfl(v[u], lane0, kWave);
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) a[u] = (own && x0 + u < nx) ? blk[(int64_t)(x0 + u) * S] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (own) acc += (double)a[u] * (double)v[u];
      }
      if (own) {
        if (it.aux == kNoSlot)
          gb.grad_b[q0 + e] = (float)acc;
        else
          gb.partial[(int64_t)it.aux * pr.d + e] = acc;
      }
    }
  }
}

// Block layout, built once per plan: words[k] = (entries of A^T row k) x
// slot(nnz(B_k)); off = their exclusive prefix sums; slot_a[perm[x]] = start
// of the block of A^T entry x, in 16-float units (-1 when B row k is empty).
__global__ void k_bw_row_words(int64_t n, const int32_t* __restrict__ atrp, const int32_t* __restrict__ brp,
                               int64_t* __restrict__ words) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    words[k] = (int64_t)(atrp[k + 1] - atrp[k]) * gb_slot(brp[k + 1] - brp[k]);
}

// one wavefront per A^T row k, lanes over its entries
__global__ void k_bw_slot_a(int64_t n, const int32_t* __restrict__ atrp, const int32_t* __restrict__ brp,
                            const int32_t* __restrict__ perm, const int64_t* __restrict__ off,
                            int32_t* __restrict__ slot_a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t k = w0; k < n; k += nw) {
    const int x0 = atrp[k], x1 = atrp[k + 1];
    const int len = brp[k + 1] - brp[k];
    const int S16 = gb_slot(len) / 16;
    const int64_t o16 = off[k] / 16;
    for (int x = x0 + lane; x < x1; x += kWave) slot_a[perm[x]] = len > 0 ? (int32_t)(o16 + (int64_t)(x - x0) * S16) : -1;
  }
}

__global__ void k_grad_b_finalize(GradBParams gb) {
  const int nrows = gb.ctr->num_split_rows;
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const SplitRow s = gb.split_rows[r];
    const int q0 = gb.pr.brp[s.row], q1 = gb.pr.brp[s.row + 1];
    for (int q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
      double acc = 0.0;
      for (int c = 0; c < s.count; ++c) acc += gb.partial[(int64_t)(s.first + c) * gb.pr.d + (q - q0)];
      gb.grad_b[q] = (float)acc;
    }
  }
}

static int check_grad_args(Plan* p, const tsspgemm_csr* A, const tsspgemm_csr* B, const tsspgemm_csr* G,
                           const void* out, const char* who) {
  int rc;
  if (!p || !p->ready || p->sr != TSSPGEMM_PLUS_TIMES_F32) {
    set_error(std::string(who) + ": needs the plus-times FP32 plan of the forward product");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (p->hash) {
    set_error(std::string(who) + ": gradients need a plan with the dense accumulator (d <= 1024)");
    return TSSPGEMM_ERR_UNSUPPORTED;
  }
  if (p->masked) {  // every product must land in pat(C) for G to be read on C's pattern
    set_error(std::string(who) + ": the forward plan was built with a mask");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if ((rc = check_csr(A, "A", true)) || (rc = check_csr(B, "B", true)) || (rc = check_csr(G, "G", true))) return rc;
  if (A->nrows != p->n || B->ncols != p->d || A->nnz != p->a_nnz || B->nnz != p->b_nnz || G->nrows != p->n ||
      G->ncols != p->d || G->nnz != p->nnz) {
    set_error(std::string(who) + ": A, B or G does not match the forward plan");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (!out) {
    set_error(std::string(who) + ": NULL output");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  return TSSPGEMM_OK;
}

static Problem plan_problem(Plan* p, const tsspgemm_csr* A, const tsspgemm_csr* B) {
  Problem pr{};
  pr.n = (int32_t)p->n;
  pr.d = (int32_t)p->d;
  pr.wp = p->wp;
  pr.arp = A->rowptr;
  pr.aci = A->colidx;
  pr.aval = A->vals;
  pr.brp = B->rowptr;
  pr.bci = B->colidx;
  pr.bval = B->vals;
  pr.bbits = (const uint32_t*)p->bbits.p;
  pr.cbits = (uint32_t*)p->cbits.p;
  pr.flops = (int64_t*)p->flops.p;
  pr.crp = p->crp;
  pr.ebnd = p->ebnd_valid ? (const int2*)p->ebnd.p : nullptr;
  return pr;
}

int light_group_lanes(int group_lanes, int64_t d, int sr);

// The first pass over A's rows (the forward plan's binned items): dL/dA dot
// products into grad_a (if non-null) and, with gather, the sampled G into
// gp.gbuf at gp.pos_a.
static int launch_grad_a_pass(Plan* p, GradAParams& gp, const tsspgemm_csr* B, bool gather, hipStream_t st) {
  // a group per B row of dot product: the smallest power of two covering the
  // mean B row length (the reduction over the group costs log2(GL) steps)
  const double mean_b = p->n > 0 ? (double)B->nnz / (double)p->n : 0.0;
  int gl = 4;
  while (gl < 64 && gl < mean_b) gl <<= 1;
  const int64_t dq = (p->d + 3) & ~3;  // strips padded so the staged records stay 16-byte aligned
  const int64_t grid = gp.n_wg_items + (p->n_wave_rows + kWavesPerBlock - 1) / kWavesPerBlock;
  const size_t lds = (size_t)kWavesPerBlock * dq * 4 + kBlock * sizeof(int4);
  const int lgl = light_group_lanes(gl, p->d, TSSPGEMM_PLUS_TIMES_I32);  // float strips: 4 bytes
  const size_t llds = (size_t)(kBlock / lgl) * dq * 4 + kBlock * sizeof(int4);
  // one workgroup per kBlock / lgl light rows: the dispatcher balances them
  // (capped at 2048 grid-striding workgroups the backward took 3.01 ms
  // instead of 2.96 at R-MAT 20 x 256)
  int64_t lgrid = (gp.n_light + (kBlock / lgl) - 1) / (kBlock / lgl);
  if (lgrid > (1 << 20)) lgrid = 1 << 20;
  const bool b8 = col_id_bytes(p->d) == 1;
  gp.pr.bcol = p->bcol.p;
#define TSS_GA_T(GLV, GA)                                                                              \
  if (b8)                                                                                              \
    k_grad_a<GLV, uint8_t, GA><<<(unsigned)grid, kBlock, lds, st>>>(gp);                               \
  else                                                                                                 \
    k_grad_a<GLV, uint16_t, GA><<<(unsigned)grid, kBlock, lds, st>>>(gp);
#define TSS_GA(GLV)                                                                                    \
  case GLV:                                                                                            \
    if (grid > 0) {                                                                                    \
      if (gather) {                                                                                    \
        TSS_GA_T(GLV, true)                                                                            \
      } else {                                                                                         \
        TSS_GA_T(GLV, false)                                                                           \
      }                                                                                                \
    }                                                                                                  \
    break;
#define TSS_GAL_T(GLV, GA)                                                                             \
  if (b8)                                                                                              \
    k_grad_a_light<GLV, uint8_t, GA><<<(unsigned)lgrid, kBlock, llds, st>>>(gp);                       \
  else                                                                                                 \
    k_grad_a_light<GLV, uint16_t, GA><<<(unsigned)lgrid, kBlock, llds, st>>>(gp);
#define TSS_GAL(GLV)                                                                                   \
  case GLV:                                                                                            \
    if (lgrid > 0) {                                                                                   \
      if (gather) {                                                                                    \
        TSS_GAL_T(GLV, true)                                                                           \
      } else {                                                                                         \
        TSS_GAL_T(GLV, false)                                                                          \
      }                                                                                                \
    }                                                                                                  \
    break;
  switch (gl) {
    TSS_GA(4) TSS_GA(8) TSS_GA(16) TSS_GA(32) TSS_GA(64)
    default: set_error("backward: bad group width"); return TSSPGEMM_ERR_INVALID_ARG;
  }
  switch (lgl) {
    TSS_GAL(4) TSS_GAL(8) TSS_GAL(16) TSS_GAL(32) TSS_GAL(64)
    default: set_error("backward: bad light group width"); return TSSPGEMM_ERR_INVALID_ARG;
  }
#undef TSS_GA
#undef TSS_GAL
#undef TSS_GA_T
#undef TSS_GAL_T
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

// Block layout of the sampled G (once per plan): B row k's blocks at
// off[k], in A^T order; slot_a[p] = start of A entry p's block in 16-float
// units.
static int ensure_sampled_positions(Plan* p, const tsspgemm_csr* AT, const tsspgemm_csr* A, const tsspgemm_csr* B,
                                    const int32_t* perm, hipStream_t st) {
  if (p->gb_pos_ready) return TSSPGEMM_OK;
  int rc;
  const int64_t n = p->n, nnz = A->nnz;
  if ((rc = p->gb_words.ensure((size_t)n * 8)) || (rc = p->gb_off.ensure((size_t)(n + 1) * 8)) ||
      (rc = p->gb_slot_a.ensure((size_t)nnz * 4)) || (rc = p->gb_scan.ensure((size_t)exscan_workspace_bytes(n))))
    return rc;
  int64_t* words = (int64_t*)p->gb_words.p;
  int64_t* off = (int64_t*)p->gb_off.p;
  const unsigned g = grid_for(n, 256) > 8192 ? 8192 : grid_for(n, 256);
  k_bw_row_words<<<g, 256, 0, st>>>(n, AT->rowptr, B->rowptr, words);
  TSS_CHECK_LAUNCH();
  if ((rc = launch_exscan_i64(words, n, off, (int64_t*)p->gb_scan.p, st))) return rc;
  // the buffer is sized by the scan's total (synchronizes once per plan)
  int64_t total = 0;
  TSS_HIP(hipMemcpyAsync(&total, off + n, 8, hipMemcpyDeviceToHost, st));
  TSS_HIP(hipStreamSynchronize(st));
  if (total / 16 > INT32_MAX) {
    set_error("backward: the sampled G needs more than 2^35 floats");
    return TSSPGEMM_ERR_UNSUPPORTED;
  }
  const unsigned gw = grid_for(n * kWave, 256) > 8192 ? 8192 : grid_for(n * kWave, 256);
  k_bw_slot_a<<<gw, 256, 0, st>>>(n, AT->rowptr, B->rowptr, perm, off, (int32_t*)p->gb_slot_a.p);
  TSS_CHECK_LAUNCH();
  p->gb_total = total;
  p->gb_pos_ready = true;
  return TSSPGEMM_OK;
}

// dL/dA and / or dL/dB (either output may be null, not both). dL/dB reads
// A^T and perm. With both, the pass over A's rows computes dL/dA and writes
// the sampled G that the dL/dB pass sums.
static int run_backward(Plan* p, const tsspgemm_csr* AT, const int32_t* perm, const tsspgemm_csr* A,
                        const tsspgemm_csr* B, const tsspgemm_csr* G, float* grad_a, float* grad_b,
                        const char* who, hipStream_t st) {
  int rc;
  if ((rc = check_grad_args(p, A, B, G, grad_a ? (const void*)grad_a : (const void*)grad_b, who))) return rc;
  if (grad_b) {
    if ((rc = check_csr(AT, "AT", false))) return rc;
    if (AT->nrows != p->n || AT->nnz != A->nnz || (A->nnz > 0 && !perm)) {
      set_error(std::string(who) + ": AT / perm do not match A");
      return TSSPGEMM_ERR_INVALID_ARG;
    }
  }
  const int64_t n = p->n, nnz = A->nnz;
  if (grad_a && nnz > 0) {
    const unsigned gz = grid_for(nnz, 256 * 4) > 8192 ? 8192 : grid_for(nnz, 256 * 4);
    k_zero_f32<<<gz, 256, 0, st>>>(grad_a, nnz);
  }
  if (grad_b && B->nnz > 0) {
    const unsigned gz = grid_for(B->nnz, 256 * 4) > 8192 ? 8192 : grid_for(B->nnz, 256 * 4);
    k_zero_f32<<<gz, 256, 0, st>>>(grad_b, B->nnz);
  }
  TSS_CHECK_LAUNCH();
  if (nnz == 0 || B->nnz == 0) return TSSPGEMM_OK;  // no products: every gradient is 0
  const bool gather = grad_b != nullptr;
  GradAParams gp{};
  gp.pr = plan_problem(p, A, B);
  gp.gci = G->colidx;
  gp.gval = (const float*)G->vals;
  gp.grad_a = grad_a;
  gp.items = (const Item*)p->num_items.p;
  gp.n_wg_items = (int32_t)(p->n_split_items + p->n_block_items);
  gp.n_heavy_records = (int32_t)(p->n_split_items + p->n_block_items + p->n_wave_rows);
  gp.n_light = (int32_t)p->n_light_rows;
  if (gather) {
    if ((rc = ensure_sampled_positions(p, AT, A, B, perm, st))) return rc;
    if ((rc = p->gb_gbuf.ensure((size_t)(p->gb_total > 0 ? p->gb_total : 1) * 4))) return rc;
    gp.gbuf = (float*)p->gb_gbuf.p;
    gp.slot_a = (const int32_t*)p->gb_slot_a.p;
  }
  if ((rc = launch_grad_a_pass(p, gp, B, gather, st))) return rc;
  if (!gather) return TSSPGEMM_OK;
  // a row of m > kGbChunk entries has ceil(m / kGbChunk) <= 2 m / kGbChunk chunks
  const int64_t chunk_cap = 2 * nnz / kGbChunk + 2;
  if ((rc = p->gb_items.ensure((size_t)(n + chunk_cap) * sizeof(Item))) ||
      (rc = p->gb_split.ensure((size_t)(n + 1) * sizeof(SplitRow))) ||
      (rc = p->gb_partial.ensure((size_t)chunk_cap * p->d * 8)) || (rc = p->gb_ctr.ensure(sizeof(Counters))))
    return rc;
  GradBParams gb{};
  gb.pr = plan_problem(p, A, B);
  gb.atrp = AT->rowptr;
  gb.grad_b = grad_b;
  gb.gbuf = (const float*)p->gb_gbuf.p;
  gb.off = (const int64_t*)p->gb_off.p;
  gb.items = (Item*)p->gb_items.p;
  gb.split_rows = (SplitRow*)p->gb_split.p;
  gb.partial = (double*)p->gb_partial.p;
  gb.ctr = (Counters*)p->gb_ctr.p;
  if (!p->gb_items_ready) {  // the work list depends only on the patterns: built once per plan
    if ((rc = launch_zero_bytes(gb.ctr, sizeof(Counters), st))) return rc;
    const unsigned g = grid_for(n, 256);
    k_gb_bin_count<<<g, 256, 0, st>>>(gb);
    k_gb_bin_scan<<<1, 1, 0, st>>>(gb.ctr);
    k_gb_bin_fill<<<g, 256, 0, st>>>(gb);
    TSS_CHECK_LAUNCH();
    p->gb_items_ready = true;
  }
  // lanes per B row: the smallest power of two covering the mean B row length
  const double mean_b = (double)B->nnz / (double)n;
  int gl = 4;
  while (gl < 64 && gl < mean_b) gl <<= 1;
  // grid-striding workgroups over the dL/dB items, eight times the resident
  // ones so that the dispatcher evens out the items (2048: 2.97 ms for the
  // backward at R-MAT 20 x 256, 16384: 2.90)
  const unsigned grid = 16384;
#define TSS_GB(GLV)                                           \
  case GLV:                                                   \
    k_grad_b_blocks<GLV><<<grid, kBlock, 0, st>>>(gb);        \
    break;
  switch (gl) {
    TSS_GB(4) TSS_GB(8) TSS_GB(16) TSS_GB(32) TSS_GB(64)
    default: set_error("backward: bad group width"); return TSSPGEMM_ERR_INVALID_ARG;
  }
#undef TSS_GB
  k_grad_b_finalize<<<1024, 256, 0, st>>>(gb);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

}  // namespace tss

extern "C" {

int tsspgemm_grad_a(tsspgemm_plan plan, const tsspgemm_csr* A, const tsspgemm_csr* B, const tsspgemm_csr* G,
                    float* grad_a, void* stream) {
  try {
    if (!grad_a) {
      tss::set_error("grad_a: NULL output");
      return TSSPGEMM_ERR_INVALID_ARG;
    }
    return tss::run_backward((tss::Plan*)plan, nullptr, nullptr, A, B, G, grad_a, nullptr, "grad_a",
                             (hipStream_t)stream);
  } catch (...) {
    tss::set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}

int tsspgemm_grad_b(tsspgemm_plan plan, const tsspgemm_csr* AT, const int32_t* at_perm, const tsspgemm_csr* A,
                    const tsspgemm_csr* B, const tsspgemm_csr* G, float* grad_b, void* stream) {
  try {
    if (!grad_b) {
      tss::set_error("grad_b: NULL output");
      return TSSPGEMM_ERR_INVALID_ARG;
    }
    return tss::run_backward((tss::Plan*)plan, AT, at_perm, A, B, G, nullptr, grad_b, "grad_b",
                             (hipStream_t)stream);
  } catch (...) {
    tss::set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}

int tsspgemm_backward(tsspgemm_plan plan, const tsspgemm_csr* AT, const int32_t* at_perm, const tsspgemm_csr* A,
                      const tsspgemm_csr* B, const tsspgemm_csr* G, float* grad_a, float* grad_b, void* stream) {
  try {
    if (!grad_a && !grad_b) {
      tss::set_error("backward: both outputs are NULL");
      return TSSPGEMM_ERR_INVALID_ARG;
    }
    return tss::run_backward((tss::Plan*)plan, AT, at_perm, A, B, G, grad_a, grad_b, "backward",
                             (hipStream_t)stream);
  } catch (...) {
    tss::set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}

}  // extern "C"
