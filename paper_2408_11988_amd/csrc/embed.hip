// Sparse force-directed embedding update (Sec. IV-B): the embedding Z (n x d,
// exactly k entries per row) is moved by attractive forces from neighbours and
// repulsive forces from negative samples, both carried by one signed n x n
// matrix A (+1 neighbour, -1 negative sample). Per row i, with s = z_i . z_j
// and sig = 1 / (1 + exp(-s)):
//   F_i = sum over stored (i, j, a) of w z_j,  w = 1 - sig (a > 0), -sig (a < 0),
// which is the TS-SpGEMM  W Z  for the weights W sampled on pat(A); then
// u = z_i + lr F_i (FP64, rounded once to FP32) and the new row keeps the k
// largest |u| (ties: lower column), sorted by column. Minibatches of rows run
// in row order; inside one, every row reads Z as it was at its start.
//
// One wavefront per work item, with z_i dense in LDS (FP32). The wavefront
// is split into P groups of GL = 64 / P lanes (GL >= k when possible); group
// g takes A entries g, g + P, ...: its lanes load z_j (coalesced), form the
// dot product with z_i, reduce it inside the group (DPP), and add w z_j into the
// group's own d-wide FP64 strip in LDS. Each group keeps U z_j rows in
// flight. The P strips are summed in group order, so every result is
// deterministic. u then replaces z_i in LDS, and the selection is a radix
// select over the 31 magnitude bits of u with ballots (lane l examines
// columns l, l + 64, ...), after which the ties at the threshold go to the
// lowest columns.
//
// Work items of a minibatch: a row with at most `chunk` A entries is one
// item, finished in place; a longer row is cut into items of `chunk`
// entries that write FP64 partial forces, and a row's partials are added in
// chunk order, then the row is updated and selected. In a small minibatch,
// whose time is its launch and its longest item, each chunk counts itself done on the row
// (a device-scope atomic between a release and an acquire fence) and the
// chunk that completes the count finishes the row, so the minibatch is one
// launch. In a large one a second kernel finishes the long rows: there the
// fences' L2 write-backs and invalidations would cost more than the launch.
// Chunk items come first; a fixed grid of wavefronts strides over the items
// (their count is read on the device, so an epoch needs no host
// synchronisation and can be captured into a graph).
//
// Minibatches ping-pong between the caller's Z and a workspace copy: batch t
// reads buffer R_t (up to date) and writes its new rows to W_t, which is stale
// only at the rows of batch t - 1; the same launch copies those rows R_t ->
// W_t.
#include "api_internal.hpp"
#include "dev_numeric.hpp"
#include "dev_reduce.hpp"

namespace tss {

constexpr int kEmbedWaves = 4;                     // wavefronts per workgroup
constexpr int64_t kEmbedFuseRows = 4096;           // minibatches up to this many rows finish long rows in place
// A entries per work item of a long row: short chunks shorten a small
// minibatch's longest dependent chain; in a large one, longer chunks write
// fewer partials
constexpr int kEmbedChunkSmall = 32, kEmbedChunkLarge = 64;

struct EmbedParams {
  int64_t n, d, k;
  const int32_t* arp;
  const int32_t* aci;
  const float* aval;
  const int32_t* rci;  // Z read buffer (up to date)
  const float* rval;
  int32_t* wci;        // Z write buffer (stale only at the previous batch's rows)
  float* wval;
  int64_t r0, nrows;   // this batch: rows [r0, r0 + nrows)
  int64_t p0, pcount;  // previous batch: rows copied R -> W
  double lr;
  const int32_t* cnt;         // chunks of each row (0: a short row)
  const int32_t* slot_off;    // exclusive scan of cnt (n + 1)
  const int32_t* slot_row;    // row of each chunk slot
  const int32_t* split_off;   // exclusive scan of (cnt > 0) (n + 1)
  const int32_t* split_list;  // rows with cnt > 0, in row order
  int32_t* done;              // chunks of each long row finished so far (zeroed at the epoch's start)
  double* partial;            // chunk slot x d partial forces
  int fuse;                   // the last chunk of a long row finishes it (no second kernel)
  int chunk;                  // A entries per work item of a long row
};

__global__ void k_embed_count(int64_t n, int chunk, const int32_t* __restrict__ arp, int32_t* __restrict__ cnt,
                              int32_t* __restrict__ split, int32_t* __restrict__ done) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int len = arp[i + 1] - arp[i];
    const int c = len > chunk ? (len + chunk - 1) / chunk : 0;
    cnt[i] = c;
    split[i] = c > 0;
    done[i] = 0;
  }
}

__global__ void k_embed_lists(int64_t n, const int32_t* __restrict__ cnt, const int32_t* __restrict__ slot_off,
                              const int32_t* __restrict__ split_off, int32_t* __restrict__ slot_row,
                              int32_t* __restrict__ split_list) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = cnt[i];
    if (c == 0) continue;
    split_list[split_off[i]] = (int32_t)i;
    for (int q = 0; q < c; ++q) slot_row[slot_off[i] + q] = (int32_t)i;
  }
}

// Lane t's share of the first 64 A entries [p0, p1) of an item.
__device__ __forceinline__ void embed_stage(const EmbedParams& ep, int p0, int p1, int lane, int& jj, float& aa) {
  jj = 0;
  aa = 0.0f;
  if (lane < p1 - p0 && lane < kWave) {
    jj = ep.aci[p0 + lane];
    aa = ep.aval[p0 + lane];
  }
}

// z_i into the wavefront's LDS row (cleared first); also clears the strips.
__device__ __forceinline__ void embed_load_zi(const EmbedParams& ep, int64_t i, float* zs, double* strips,
                                              int64_t nstrip, int lane) {
  wave_sync();
  for (int64_t c = lane; c < ep.d; c += kWave) zs[c] = 0.0f;
  for (int64_t c = lane; c < nstrip; c += kWave) strips[c] = 0.0;
  wave_sync();
  for (int64_t t = lane; t < ep.k; t += kWave) {
    const int32_t c = ep.rci[i * ep.k + t];
    if ((uint32_t)c < (uint64_t)ep.d) zs[c] = ep.rval[i * ep.k + t];
  }
  wave_sync();
}

// Forces of A entries [p0, p1) of one row into the group strips.
// The first 64 entries arrive staged (jj0, aa0: lane t holds entry p0 + t),
// loaded by the caller before z_i so that both loads are in flight at once.
template <int P, int KPL, int U>
__device__ __forceinline__ void embed_accumulate(const EmbedParams& ep, int p0, int p1, int jj0, float aa0,
                                                 const float* zs, double* myF, int lane, int g, int gl) {
  constexpr int GL = kWave / P;
  const int64_t d = ep.d, k = ep.k;
  for (int base = p0; base < p1; base += kWave) {
    const int nb = min(kWave, p1 - base);
    int jj = jj0;
    float aa = aa0;
    if (base != p0) {
      jj = 0;
      aa = 0.0f;
      if (lane < nb) {
        jj = ep.aci[base + lane];
        aa = ep.aval[base + lane];
      }
    }
    for (int s = 0; s < nb; s += P * U) {  // uniform trip count: shuffles see every lane
      float a[U];
      int32_t cc[U][KPL];
      float vv[U][KPL];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = s + u * P + g;
        const int j = __shfl(jj, e < nb ? e : 0, kWave);
        a[u] = __shfl(aa, e < nb ? e : 0, kWave);
        const bool live = e < nb && (uint32_t)j < (uint64_t)ep.n;
#pragma unroll
        for (int q = 0; q < KPL; ++q) {
          const int64_t t = (int64_t)q * GL + gl;
          cc[u][q] = -1;
          vv[u][q] = 0.0f;
          if (live && t < k) {
            cc[u][q] = ep.rci[(int64_t)j * k + t];
            vv[u][q] = ep.rval[(int64_t)j * k + t];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        double dot = 0.0;
#pragma unroll
        for (int q = 0; q < KPL; ++q)
          if ((uint32_t)cc[u][q] < (uint64_t)d) dot += (double)zs[cc[u][q]] * (double)vv[u][q];
        dot = group_sum_f64<GL>(dot);
        const double sig = 1.0 / (1.0 + exp(-dot));
        const double w = a[u] > 0.0f ? 1.0 - sig : (a[u] < 0.0f ? -sig : 0.0);
#pragma unroll
        for (int q = 0; q < KPL; ++q)
          if ((uint32_t)cc[u][q] < (uint64_t)d) myF[cc[u][q]] += w * (double)vv[u][q];
      }
    }
  }
  wave_sync();
}

// New row i from u (the wavefront's d-wide LDS row `us`): the k largest |u|,
// ties to the lowest columns, written sorted by column at row i of W. Lane
// l examines columns l, l + 64, ...
__device__ __forceinline__ void embed_select_write(const EmbedParams& ep, int64_t i, const float* us, int lane) {
  const int64_t d = ep.d, k = ep.k;
  const int M = (int)((d + kWave - 1) / kWave);
  // T: bits fixed from the top while #{c : |u_c| >= T} >= k holds. The search
  // ends at the k-th largest key, or earlier once exactly k keys are >= T:
  // those k keys are then the k largest, with no tie to break (d == k: all).
  uint32_t T = 0;
  if (d > k && M <= 2) {  // d <= 128: the lane's two keys stay in registers
    const int64_t c1 = kWave + lane;
    const uint32_t k0 = lane < d ? __float_as_uint(us[lane]) & 0x7fffffffu : 0u;
    const uint32_t k1 = c1 < d ? __float_as_uint(us[c1]) & 0x7fffffffu : 0u;
    const bool in0 = lane < d, in1 = c1 < d;
    for (int b = 30; b >= 0; --b) {
      const uint32_t cand = T | (1u << b);
      const int cnt = __popcll(__ballot(in0 && k0 >= cand)) + __popcll(__ballot(in1 && k1 >= cand));
      if (cnt >= k) {
        T = cand;
        if (cnt == k) break;
      }
    }
  } else if (d > k) {
    for (int b = 30; b >= 0; --b) {
      const uint32_t cand = T | (1u << b);
      int cnt = 0;
      for (int m = 0; m < M; ++m) {
        const int64_t c = (int64_t)m * kWave + lane;
        cnt += __popcll(__ballot(c < d && (__float_as_uint(us[c < d ? c : 0]) & 0x7fffffffu) >= cand));
      }
      if (cnt >= k) {
        T = cand;
        if (cnt == k) break;
      }
    }
  }
  int above = 0;  // #{key > T} <= k
  for (int m = 0; m < M; ++m) {
    const int64_t c = (int64_t)m * kWave + lane;
    above += __popcll(__ballot(c < d && (__float_as_uint(us[c < d ? c : 0]) & 0x7fffffffu) > T));
  }
  const int need = (int)k - above;  // ties at T taken from the lowest columns
  int eq_before = 0, written = 0;
  const int64_t out = i * k;
  for (int m = 0; m < M; ++m) {
    const int64_t c = (int64_t)m * kWave + lane;
    const bool in = c < d;
    const float u = us[in ? c : 0];
    const uint32_t key = __float_as_uint(u) & 0x7fffffffu;
    const uint64_t eq = __ballot(in && key == T);
    const bool sel = in && (key > T || (key == T && eq_before + lanes_below(eq) < need));
    const uint64_t sm = __ballot(sel);
    if (sel) {
      const int64_t pos = out + written + lanes_below(sm);
      ep.wci[pos] = (int32_t)c;
      ep.wval[pos] = u;
    }
    eq_before += __popcll(eq);
    written += __popcll(sm);
  }
}

// A long row once all its chunks are written: partial forces added in chunk
// order (eight loads issued before their sums), u = z_i + lr F into the
// wavefront's LDS row `zs` (which holds z_i), then the selection.
__device__ __forceinline__ void embed_finish_long(const EmbedParams& ep, int64_t i, float* zs, int lane) {
  const int64_t d = ep.d;
  const int nc = ep.cnt[i];
  const double* part = ep.partial + (int64_t)ep.slot_off[i] * d;
  for (int64_t col = lane; col < d; col += kWave) {  // each lane its own columns
    double f = 0.0;
    int c = 0;
    for (; c + 8 <= nc; c += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = part[(int64_t)(c + q) * d + col];
#pragma unroll
      for (int q = 0; q < 8; ++q) f += v[q];
    }
    for (; c < nc; ++c) f += part[(int64_t)c * d + col];
    zs[col] = (float)((double)zs[col] + ep.lr * f);
  }
  wave_sync();
  embed_select_write(ep, i, zs, lane);
}

// Items of one minibatch (chunks of long rows, then short rows) and the
// copy of the previous minibatch's rows.
template <int P, int KPL>
__global__ __launch_bounds__(kEmbedWaves * kWave) void k_embed_main(EmbedParams ep) {
  extern __shared__ __align__(16) unsigned char embed_smem[];
  constexpr int GL = kWave / P;
  constexpr int U = KPL >= 4 ? 1 : 4 / KPL;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;  // wavefronts in this workgroup
  const int g = lane / GL, gl = lane % GL;
  const int64_t d = ep.d, k = ep.k;
  double* strips = reinterpret_cast<double*>(embed_smem) + (int64_t)wave * P * d;
  float* zs = reinterpret_cast<float*>(embed_smem + (size_t)nw * P * d * sizeof(double)) + wave * d;
  const int64_t gw = (int64_t)blockIdx.x * nw + wave;
  const int64_t tw = (int64_t)gridDim.x * nw;

  for (int64_t q = gw; q < ep.pcount; q += tw) {
    const int64_t r = (ep.p0 + q) * k;
    for (int64_t t = lane; t < k; t += kWave) {
      ep.wci[r + t] = ep.rci[r + t];
      ep.wval[r + t] = ep.rval[r + t];
    }
  }
  const int32_t s0 = ep.slot_off[ep.r0], s1 = ep.slot_off[ep.r0 + ep.nrows];
  const int64_t nch = s1 - s0;
  for (int64_t it = gw; it < nch + ep.nrows; it += tw) {
    if (it < nch) {
      const int32_t slot = s0 + (int32_t)it;
      const int64_t i = ep.slot_row[slot];
      const int c = slot - ep.slot_off[i];
      const int p0 = ep.arp[i] + c * ep.chunk;
      const int p1 = min(ep.arp[i + 1], p0 + ep.chunk);
      int jj0;
      float aa0;
      embed_stage(ep, p0, p1, lane, jj0, aa0);
      embed_load_zi(ep, i, zs, strips, P * d, lane);
      embed_accumulate<P, KPL, U>(ep, p0, p1, jj0, aa0, zs, strips + (int64_t)g * d, lane, g, gl);
      for (int64_t col = lane; col < d; col += kWave) {
        double f = 0.0;
#pragma unroll
        for (int gg = 0; gg < P; ++gg) f += strips[(int64_t)gg * d + col];
        ep.partial[(int64_t)slot * d + col] = f;
      }
      if (!ep.fuse) continue;
      // publish this chunk's partials, then count it; the row's last chunk
      // (in completion order) sees every partial after its acquire
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      int prev = 0;
      if (lane == 0) prev = __hip_atomic_fetch_add(ep.done + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      prev = __shfl(prev, 0, kWave);
      if (prev != ep.cnt[i] - 1) continue;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      embed_finish_long(ep, i, zs, lane);
    } else {
      const int64_t i = ep.r0 + (it - nch);
      if (ep.cnt[i] > 0) continue;  // a long row: finished by its last chunk or the finalize kernel
      const int p0 = ep.arp[i], p1 = ep.arp[i + 1];
      int jj0;
      float aa0;
      embed_stage(ep, p0, p1, lane, jj0, aa0);
      embed_load_zi(ep, i, zs, strips, P * d, lane);
      embed_accumulate<P, KPL, U>(ep, p0, p1, jj0, aa0, zs, strips + (int64_t)g * d, lane, g, gl);
      for (int64_t col = lane; col < d; col += kWave) {  // u replaces z_i in LDS (each lane its own columns)
        double f = 0.0;
#pragma unroll
        for (int gg = 0; gg < P; ++gg) f += strips[(int64_t)gg * d + col];
        zs[col] = (float)((double)zs[col] + ep.lr * f);
      }
      wave_sync();
      embed_select_write(ep, i, zs, lane);
    }
  }
}

// Long rows of one minibatch: partial forces added in chunk order, update,
// selection.
__global__ __launch_bounds__(kEmbedWaves * kWave) void k_embed_finalize(EmbedParams ep) {
  extern __shared__ __align__(16) unsigned char embed_smem[];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int64_t d = ep.d;
  float* zs = reinterpret_cast<float*>(embed_smem) + wave * d;
  const int64_t gw = (int64_t)blockIdx.x * kEmbedWaves + wave;
  const int64_t tw = (int64_t)gridDim.x * kEmbedWaves;
  const int32_t m0 = ep.split_off[ep.r0], m1 = ep.split_off[ep.r0 + ep.nrows];
  for (int64_t q = gw; q < m1 - m0; q += tw) {
    const int64_t i = ep.split_list[m0 + q];
    embed_load_zi(ep, i, zs, nullptr, 0, lane);
    embed_finish_long(ep, i, zs, lane);
  }
}

// Groups per wavefront: GL = 64 / P lanes should cover the k entries of a z
// row; the P FP64 strips of the four wavefronts must fit 64 KB with z_i.
static int embed_groups(int64_t d, int64_t k) {
  int P = 1;
  while (P < 8 && kWave / (2 * P) >= k) P <<= 1;
  while (P > 1 && (int64_t)kEmbedWaves * (8 * P * d + 4 * d) > 65536) P >>= 1;
  return P;
}

static size_t embed_lds(int64_t d, int P, int nw) { return (size_t)nw * (8 * (size_t)P * d + 4 * (size_t)d); }

template <int P, int KPL>
static int launch_embed_t(const EmbedParams& ep, unsigned grid, int nw, hipStream_t st) {
  k_embed_main<P, KPL><<<grid, nw * kWave, embed_lds(ep.d, P, nw), st>>>(ep);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

static int launch_embed(const EmbedParams& ep, int P, hipStream_t st) {
  const int64_t k = ep.k;
  // wavefronts: two per row of the minibatch (room for the chunks of its long
  // rows; further items stride), at least 256 and at most 8192
  int64_t waves = 2 * ep.nrows > ep.pcount ? 2 * ep.nrows : ep.pcount;
  if (waves < 256) waves = 256;
  if (waves > 8192) waves = 8192;
  // a small minibatch spreads its wavefronts one per workgroup over the CUs
  const int nw = ep.fuse ? 1 : kEmbedWaves;
  const unsigned grid = (unsigned)((waves + nw - 1) / nw);
  int rc;
  switch (P) {
    case 8: rc = launch_embed_t<8, 1>(ep, grid, nw, st); break;
    case 4: rc = launch_embed_t<4, 1>(ep, grid, nw, st); break;
    case 2: rc = launch_embed_t<2, 1>(ep, grid, nw, st); break;
    default:
      if (k <= 64) rc = launch_embed_t<1, 1>(ep, grid, nw, st);
      else if (k <= 128) rc = launch_embed_t<1, 2>(ep, grid, nw, st);
      else if (k <= 256) rc = launch_embed_t<1, 4>(ep, grid, nw, st);
      else if (k <= 512) rc = launch_embed_t<1, 8>(ep, grid, nw, st);
      else rc = launch_embed_t<1, 16>(ep, grid, nw, st);
  }
  if (rc || ep.fuse) return rc;
  const unsigned fgrid = grid < 256 ? grid : 256;
  k_embed_finalize<<<fgrid, kEmbedWaves * kWave, (size_t)kEmbedWaves * 4 * ep.d, st>>>(ep);
  TSS_CHECK_LAUNCH();
  return TSSPGEMM_OK;
}

static int run_embed_epoch(const tsspgemm_csr* A, int64_t d, int64_t k, int32_t* zci, float* zval, float lr,
                           int64_t batch, int64_t row_begin, int64_t row_end, hipStream_t st) {
  int rc;
  if ((rc = check_csr(A, "A", true))) return rc;
  if (A->nrows != A->ncols) {
    set_error("embed: A must be square (n x n)");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  const int64_t n = A->nrows;
  if (d < 1 || k < 1 || k > d || batch < 1 || row_begin < 0 || row_begin > row_end || row_end > n ||
      (n > 0 && (!zci || !zval))) {
    set_error("embed: need 1 <= k <= d, batch >= 1, 0 <= row_begin <= row_end <= n and Z buffers");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (d > kMaxDenseD) {
    set_error("embed: d > 1024");
    return TSSPGEMM_ERR_UNSUPPORTED;
  }
  if (row_begin == row_end) return TSSPGEMM_OK;
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
  const size_t zbytes = (size_t)n * (size_t)k * 4;
  const int chunk = batch <= kEmbedFuseRows ? kEmbedChunkSmall : kEmbedChunkLarge;
  // a row of len > chunk entries has ceil(len / chunk) < 2 len / chunk chunks
  const int64_t slot_cap = 2 * A->nnz / chunk + 1;
  if ((rc = p->em_ci.ensure(zbytes)) || (rc = p->em_val.ensure(zbytes)) ||
      (rc = p->em_cnt.ensure((size_t)n * 4)) || (rc = p->em_split.ensure((size_t)n * 4)) ||
      (rc = p->em_done.ensure((size_t)n * 4)) ||
      (rc = p->em_slot_off.ensure((size_t)(n + 1) * 4)) || (rc = p->em_split_off.ensure((size_t)(n + 1) * 4)) ||
      (rc = p->em_slot_row.ensure((size_t)slot_cap * 4)) || (rc = p->em_split_list.ensure((size_t)n * 4)) ||
      (rc = p->em_partial.ensure((size_t)slot_cap * d * 8)) ||
      (rc = p->em_scan.ensure((size_t)exscan_workspace_bytes(n))))
    return rc;
  int32_t* xci = (int32_t*)p->em_ci.p;
  float* xval = (float*)p->em_val.p;
  EmbedParams ep{};
  ep.n = n;
  ep.d = d;
  ep.k = k;
  ep.arp = A->rowptr;
  ep.aci = A->colidx;
  ep.aval = (const float*)A->vals;
  ep.lr = (double)lr;
  ep.cnt = (const int32_t*)p->em_cnt.p;
  ep.slot_off = (const int32_t*)p->em_slot_off.p;
  ep.slot_row = (const int32_t*)p->em_slot_row.p;
  ep.split_off = (const int32_t*)p->em_split_off.p;
  ep.split_list = (const int32_t*)p->em_split_list.p;
  ep.done = (int32_t*)p->em_done.p;
  ep.chunk = chunk;
  ep.partial = (double*)p->em_partial.p;
  {
    const unsigned g = grid_for(n, 256) > 4096 ? 4096 : grid_for(n, 256);
    k_embed_count<<<g, 256, 0, st>>>(n, chunk, A->rowptr, (int32_t*)p->em_cnt.p, (int32_t*)p->em_split.p,
                                     (int32_t*)p->em_done.p);
    TSS_CHECK_LAUNCH();
    if ((rc = launch_exscan_i32((const int32_t*)p->em_cnt.p, n, (int32_t*)p->em_slot_off.p, (int64_t*)p->em_scan.p,
                                st)) ||
        (rc = launch_exscan_i32((const int32_t*)p->em_split.p, n, (int32_t*)p->em_split_off.p,
                                (int64_t*)p->em_scan.p, st)))
      return rc;
    k_embed_lists<<<g, 256, 0, st>>>(n, ep.cnt, ep.slot_off, ep.split_off, (int32_t*)p->em_slot_row.p,
                                     (int32_t*)p->em_split_list.p);
    TSS_CHECK_LAUNCH();
  }
  TSS_HIP(hipMemcpyAsync(xci, zci, zbytes, hipMemcpyDeviceToDevice, st));
  TSS_HIP(hipMemcpyAsync(xval, zval, zbytes, hipMemcpyDeviceToDevice, st));
  const int P = embed_groups(d, k);
  int64_t t = 0, prev0 = 0, prevn = 0;
  for (int64_t r0 = row_begin; r0 < row_end; r0 += batch, ++t) {
    const bool even = (t % 2) == 0;  // even batches read the caller's Z and write the workspace
    ep.rci = even ? zci : xci;
    ep.rval = even ? zval : xval;
    ep.wci = even ? xci : zci;
    ep.wval = even ? xval : zval;
    ep.r0 = r0;
    ep.nrows = (row_end - r0) < batch ? (row_end - r0) : batch;
    ep.p0 = prev0;
    ep.pcount = t > 0 ? prevn : 0;
    ep.fuse = ep.nrows <= kEmbedFuseRows;
    if ((rc = launch_embed(ep, P, st))) return rc;
    prev0 = r0;
    prevn = ep.nrows;
  }
  if ((t - 1) % 2 == 0) {  // the last batch wrote the workspace: bring its rows back
    TSS_HIP(hipMemcpyAsync(zci + prev0 * k, xci + prev0 * k, (size_t)prevn * k * 4, hipMemcpyDeviceToDevice, st));
    TSS_HIP(hipMemcpyAsync(zval + prev0 * k, xval + prev0 * k, (size_t)prevn * k * 4, hipMemcpyDeviceToDevice, st));
  }
  return TSSPGEMM_OK;
}

}  // namespace tss

extern "C" int tsspgemm_embed_epoch(const tsspgemm_csr* A, int64_t d, int64_t k, int32_t* z_colidx, float* z_vals,
                                    float lr, int64_t batch_rows, int64_t row_begin, int64_t row_end, void* stream) {
  try {
    return tss::run_embed_epoch(A, d, k, z_colidx, z_vals, lr, batch_rows, row_begin, row_end, (hipStream_t)stream);
  } catch (...) {
    tss::set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}
