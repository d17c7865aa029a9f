// Multi-source BFS by repeated masked Boolean TS-SpGEMM (Sec. IV-A,
// Algorithm 3): N = A F over (AND, OR), F = N \ S, S = S v N, until F is empty.
//
// Every matrix of the loop is kept as a bitmap of d bits per row (d <= 1024):
// F (the frontier, the "B" of the multiply), S (visited, the complement
// mask) and N. One iteration is the symbolic pass of the library (bitmap
// accumulator, row binning of A done once) with two row filters that do not
// change the result: A entries whose frontier row is empty are skipped (a
// 1-bit-per-row summary of F), rows whose unvisited columns all belong to
// sources whose frontier is already empty are skipped (a d-bit "active" word
// mask), and a row stops reading neighbours once its accumulator holds every
// column still open to it (later ones could only add masked bits). The
// masked product is directly N \ S, i.e. the next frontier.
// Levels are written once, at the end, from the kept frontiers N_0..N_T: a
// lane owns 4 consecutive columns of a row (one 16-byte store), so every
// store is coalesced, and never-reached pairs get -1 in the same pass.
#include <string>
#include <type_traits>
#include <vector>

#include "api_internal.hpp"

namespace tss {

constexpr int kBfsUpdateBlocks = 2048;  // fixed grid of the frontier update

// N_0: bit j of row sources[j]; a source outside [0, n) sets the error flag.
__global__ void k_bfs_seed(const int32_t* __restrict__ src, int32_t d, int64_t n, int wp, uint32_t* __restrict__ n0,
                           int64_t* __restrict__ bad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  const int32_t v = src[j];
  if (v < 0 || v >= n) {
    atomicOr((unsigned long long*)bad, 1ull);
    return;
  }
  atomicOr(&n0[(int64_t)v * wp + (j >> 5)], 1u << (j & 31));
}

// S |= N, the non-empty-row summary of N (fnz: bit r of word i >> 5 = row i
// of N has a bit), and per workgroup the OR of N's words by column word and
// the number of set bits. A fixed grid strides over tiles of 256 V / wp rows,
// V = min(4, wp) words per lane (one 4-, 8- or 16-byte load): thread t
// always holds the same V word columns, so every load is coalesced; the
// wp / V lanes of a row OR their words with shuffles for its summary bit, and
// a tile's summary words (32 rows each) are gathered in LDS.
template <int V>
__global__ __launch_bounds__(256) void k_bfs_update(int64_t n, int wp, const uint32_t* __restrict__ N,
                                                    uint32_t* __restrict__ S, uint32_t* __restrict__ fnz,
                                                    uint32_t* __restrict__ part_or, int64_t* __restrict__ part_cnt) {
  using Vec = typename std::conditional<V == 4, uint4, typename std::conditional<V == 2, uint2, uint32_t>::type>::type;
  constexpr int kMaxTileWords = 256 * V / 32;  // summary words per tile (at most 32)
  __shared__ uint32_t sor[32];
  __shared__ uint32_t sfnz[kMaxTileWords];
  __shared__ unsigned long long scnt;
  const int t = threadIdx.x;
  if (t < 32) sor[t] = 0u;
  if (t < kMaxTileWords) sfnz[t] = 0u;
  if (t == 0) scnt = 0ull;
  __syncthreads();
  const int lpr = wp / V;                  // lanes per row
  const int w0 = (t % lpr) * V;            // this thread's first word column
  const int rows = 256 / lpr;              // rows per tile
  const int64_t ntiles = (n + rows - 1) / rows;
  uint32_t wor[V];
#pragma unroll
  for (int v = 0; v < V; ++v) wor[v] = 0u;
  long long cnt = 0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int r = t / lpr;
    const int64_t row = tile * rows + r;
    uint32_t x[V];
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = 0u;
    if (row < n) {
      const Vec xv = *reinterpret_cast<const Vec*>(N + row * wp + w0);
      if constexpr (V == 4) {
        x[0] = xv.x; x[1] = xv.y; x[2] = xv.z; x[3] = xv.w;
      } else if constexpr (V == 2) {
        x[0] = xv.x; x[1] = xv.y;
      } else {
        x[0] = xv;
      }
    }
    uint32_t any = 0u;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      any |= x[v];
      wor[v] |= x[v];
      cnt += __popc(x[v]);
    }
    if (any) {
      Vec* sp = reinterpret_cast<Vec*>(S + row * wp + w0);
      Vec sv = *sp;
      if constexpr (V == 4) {
        sv.x |= x[0]; sv.y |= x[1]; sv.z |= x[2]; sv.w |= x[3];
      } else if constexpr (V == 2) {
        sv.x |= x[0]; sv.y |= x[1];
      } else {
        sv |= x[0];
      }
      *sp = sv;
    }
    for (int o = 1; o < lpr; o <<= 1) any |= shfl_xor_u32(any, o);
    if (t % lpr == 0 && any) atomicOr(&sfnz[r >> 5], 1u << (r & 31));
    __syncthreads();
    const int tw = (rows + 31) / 32;
    if (t < tw) {
      const int64_t fw = tile * rows / 32 + t;  // rows is a multiple of 32
      if (fw * 32 < n) fnz[fw] = sfnz[t];
      sfnz[t] = 0u;
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < V; ++v)
    if (wor[v]) atomicOr(&sor[w0 + v], wor[v]);
  const long long wsum = wave_sum_i64(cnt);
  if ((t & (kWave - 1)) == 0 && wsum) atomicAdd(&scnt, (unsigned long long)wsum);
  __syncthreads();
  if (t < wp) part_or[(int64_t)blockIdx.x * wp + t] = sor[t];
  if (t == 0) part_cnt[blockIdx.x] = (int64_t)scnt;
}

// One workgroup: OR of the partial column masks -> active, sum -> count.
__global__ __launch_bounds__(1024) void k_bfs_reduce(int64_t nblocks, int wp, const uint32_t* __restrict__ part_or,
                                                     const int64_t* __restrict__ part_cnt,
                                                     uint32_t* __restrict__ active, int64_t* __restrict__ count) {
  __shared__ uint32_t sor[32];
  __shared__ unsigned long long scnt;
  if (threadIdx.x < 32) sor[threadIdx.x] = 0u;
  if (threadIdx.x == 0) scnt = 0ull;
  __syncthreads();
  unsigned long long c = 0;
  for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) c += (unsigned long long)part_cnt[b];
  for (int64_t t = threadIdx.x; t < nblocks * wp; t += blockDim.x) {
    const uint32_t x = part_or[t];
    if (x) atomicOr(&sor[t % wp], x);
  }
  atomicAdd(&scnt, c);
  __syncthreads();
  if (threadIdx.x < wp) active[threadIdx.x] = sor[threadIdx.x];
  if (threadIdx.x == 0) *count = (int64_t)scnt;
}

// level[i*d + j] = t for the frontier N_t holding bit j of row i, else -1.
// A lane owns 4 consecutive columns (one 16-byte store when d is a multiple of
// 4), a wavefront 256 columns of one row; work units (row, 256-column chunk)
// are walked grid-stride. The frontier loads of one lane are independent (no
// early exit), so they are all in flight together; the frontiers are visited
// from last to first so the earliest one holding the bit wins.
__global__ __launch_bounds__(256) void k_bfs_levels(int64_t n, int32_t d, int wp, int32_t nfront,
                                                    const uint32_t* const* __restrict__ fronts,
                                                    int32_t* __restrict__ levels) {
  const int lane = threadIdx.x & 63;
  const int nch = (d + 255) >> 8;
  const int64_t units = n * nch;
  const int64_t wstride = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const bool vec = (d & 3) == 0 && ((uintptr_t)levels & 15) == 0;
  for (int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; u < units; u += wstride) {
    const int64_t row = u / nch;
    const int j0 = ((int)(u % nch) << 8) + 4 * lane;  // first of this lane's 4 columns
    if (j0 >= d) continue;
    const int64_t word = row * wp + (j0 >> 5);
    const int sh = j0 & 31;  // the 4 bits j0..j0+3 sit in one word (j0 is a multiple of 4)
    int l0 = -1, l1 = -1, l2 = -1, l3 = -1;
#pragma unroll 4
    for (int t = nfront - 1; t >= 0; --t) {
      const uint32_t x = fronts[t][word] >> sh;
      l0 = (x & 1u) ? t : l0;
      l1 = (x & 2u) ? t : l1;
      l2 = (x & 4u) ? t : l2;
      l3 = (x & 8u) ? t : l3;
    }
    int32_t* out = levels + row * d + j0;
    if (vec) {
      typedef int v4i __attribute__((ext_vector_type(4)));
      const v4i v = {l0, l1, l2, l3};
      __builtin_nontemporal_store(v, reinterpret_cast<v4i*>(out));  // streamed out, never re-read here
    } else {
      const int m = d - j0 < 4 ? d - j0 : 4;
      out[0] = l0;
      if (m > 1) out[1] = l1;
      if (m > 2) out[2] = l2;
      if (m > 3) out[3] = l3;
    }
  }
}

// The same levels when d is a multiple of 32, a lane per bitmap word: the
// lane loads its word of every frontier (a wavefront reads 256 contiguous
// bytes per frontier) and folds the frontiers from last to first into bit
// planes of the level (five planes: up to 32 frontiers) and an any-frontier
// mask, so the earliest frontier holding a bit wins, as above. The 64 words
// of a wavefront are 8 KB of levels, contiguous (word q holds columns
// 32 q .. 32 q + 31 of the flattened n x d array): in store round c, lane l
// takes the planes of word 8 c + l / 8 by shuffle and writes its 4 levels
// at 16 l bytes into the round's kilobyte, so every store is coalesced.
__global__ __launch_bounds__(256) void k_bfs_levels_words(int64_t n, int32_t d, int wp, int32_t nfront,
                                                          const uint32_t* const* __restrict__ fronts,
                                                          int32_t* __restrict__ levels) {
  const int wpd = d >> 5;  // words of a row that hold columns
  const int64_t words = n * wpd;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t q0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * kWave; q0 < words;
       q0 += nwaves * kWave) {
    const int64_t q = q0 + lane;
    uint32_t pl0 = 0, pl1 = 0, pl2 = 0, pl3 = 0, pl4 = 0, any = 0;
    if (q < words) {
      const int64_t row = q / wpd;
      const int64_t word = row * wp + (q - row * wpd);
#pragma unroll 4
      for (int t = nfront - 1; t >= 0; --t) {
        const uint32_t x = fronts[t][word];
        any |= x;
        pl0 = (pl0 & ~x) | ((t & 1) ? x : 0u);
        pl1 = (pl1 & ~x) | ((t & 2) ? x : 0u);
        pl2 = (pl2 & ~x) | ((t & 4) ? x : 0u);
        pl3 = (pl3 & ~x) | ((t & 8) ? x : 0u);
        pl4 = (pl4 & ~x) | ((t & 16) ? x : 0u);
      }
    }
    typedef int v4i __attribute__((ext_vector_type(4)));
    const int sh = 4 * (lane & 7);  // this lane's 4 bits of the source word
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int src = 8 * c + (lane >> 3);
      const uint32_t a = shfl_u32(any, src), b0 = shfl_u32(pl0, src), b1 = shfl_u32(pl1, src);
      const uint32_t b2 = shfl_u32(pl2, src), b3 = shfl_u32(pl3, src), b4 = shfl_u32(pl4, src);
      if (q0 + src >= words) continue;
      v4i v;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = sh + e;
        const int l = (int)(((b0 >> j) & 1u) | (((b1 >> j) & 1u) << 1) | (((b2 >> j) & 1u) << 2) |
                            (((b3 >> j) & 1u) << 3) | (((b4 >> j) & 1u) << 4));
        v[e] = ((a >> j) & 1u) ? l : -1;
      }
      // streamed out, never re-read here
      __builtin_nontemporal_store(v, reinterpret_cast<v4i*>(levels + (q0 + src) * 32 + sh));
    }
  }
}

struct BfsWork {
  DevBuf S, fnz, active, part_or, part_cnt, count, fronts_dev;
  std::vector<DevBuf> fronts;
  int64_t* host_count = nullptr;  // pinned: [nnz of the frontier, bad-source flag]
  ~BfsWork() {
    if (host_count) (void)hipHostFree(host_count);
  }
};

// The BFS workspace of a device (counters, item list, visited set, one
// frontier bitmap per level), kept between calls: the frontiers alone are
// levels x n x wp words, which would otherwise be allocated and freed by
// every call. Calls on one device hold its mutex for the whole search; the
// plan's events order them across streams.
struct BfsState {
  std::mutex mu;
  Plan p;
  BfsWork w;
};
static std::mutex g_bfs_mu;
static BfsState* g_bfs[64];

static BfsState* bfs_state(int dev) {
  std::lock_guard<std::mutex> lk(g_bfs_mu);
  if (dev < 0 || dev >= 64) return nullptr;
  if (!g_bfs[dev]) g_bfs[dev] = new (std::nothrow) BfsState();
  return g_bfs[dev];
}

static int run_msbfs(const tsspgemm_csr* A, const int32_t* sources, int32_t d, int32_t* levels,
                     int32_t* iterations, int64_t* frontier_nnz, int32_t capacity, hipStream_t st) {
  int rc;
  if ((rc = check_csr(A, "A", false))) return rc;
  if (A->nrows != A->ncols) {
    set_error("A must be square (n x n)");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (d < 1 || d > kMaxDenseD) {
    set_error("msbfs: d must be in [1, 1024]");
    return d < 1 ? TSSPGEMM_ERR_INVALID_ARG : TSSPGEMM_ERR_UNSUPPORTED;
  }
  if (!sources || !levels || !iterations) {
    set_error("msbfs: NULL argument");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  const int64_t n = A->nrows;
  const int wp = bitmap_words(d);
  int dev = 0;
  TSS_HIP(hipGetDevice(&dev));
  BfsState* state = bfs_state(dev);
  if (!state) {
    set_error("msbfs: no workspace for this device");
    return TSSPGEMM_ERR_NOMEM;
  }
  std::lock_guard<std::mutex> lk(state->mu);
  StreamOrder so(&state->p, st);
  if (so.rc) return so.rc;
  Plan& p = state->p;
  BfsWork& w = state->w;
  if (!w.host_count) TSS_HIP(hipHostMalloc((void**)&w.host_count, 2 * sizeof(int64_t), hipHostMallocDefault));
  p.n = n;
  p.d = d;
  p.wp = wp;
  tsspgemm_tuning tn{};
  tsspgemm_csr bdummy{n, d, 0, A->rowptr, nullptr, nullptr};
  resolve_tuning(nullptr, &bdummy, &tn);
  tn.sym_split_nnz = sym_split_default(wp, true);  // heavy items stop once their open columns are covered
  const int64_t sym_cap = n + A->nnz / tn.sym_split_nnz + 2;
  const int upd_v = wp < 4 ? wp : 4;                        // words per lane in k_bfs_update
  const int64_t upd_rows = 256 / (wp / upd_v);              // rows per tile
  const int64_t ntiles = (n + upd_rows - 1) / upd_rows;
  const int64_t nblk = ntiles < kBfsUpdateBlocks ? ntiles : kBfsUpdateBlocks;  // workgroups of k_bfs_update
  if ((rc = p.ctr.ensure(sizeof(Counters))) || (rc = p.flops.ensure((size_t)n * 8)) ||
      (rc = p.sym_items.ensure((size_t)sym_cap * sizeof(Item))) || (rc = w.S.ensure((size_t)n * wp * 4)) ||
      (rc = w.fnz.ensure((size_t)(n / 32 + 4) * 4)) || (rc = w.active.ensure(32 * 4)) ||
      (rc = w.part_or.ensure((size_t)(nblk + 1) * wp * 4)) || (rc = w.part_cnt.ensure((size_t)(nblk + 1) * 8)) ||
      (rc = w.count.ensure(16)))
    return rc;
  if (!p.host_ctr) TSS_HIP(hipHostMalloc((void**)&p.host_ctr, sizeof(Counters), hipHostMallocDefault));
  if (validate_enabled() && (rc = validate_on_device(A, "A", (Counters*)p.ctr.p, p.host_ctr, st))) return rc;
  Counters* ctr = (Counters*)p.ctr.p;
  Problem pr{};
  pr.n = (int32_t)n;
  pr.d = d;
  pr.wp = wp;
  pr.arp = A->rowptr;
  pr.aci = A->colidx;
  pr.flops = (int64_t*)p.flops.p;
  if ((rc = launch_zero_bytes(ctr, sizeof(Counters), st))) return rc;
  if ((rc = launch_sym_bin(pr, tn.sym_split_nnz, (Item*)p.sym_items.p, ctr, st, false, kSlotRowMaxBfs))) return rc;

  size_t nf = 0;  // frontiers of this call: w.fronts[0, nf)
  auto new_front = [&](uint32_t** out) -> int {
    if (nf == w.fronts.size()) w.fronts.emplace_back();
    int r = w.fronts[nf].ensure((size_t)n * wp * 4);
    *out = (uint32_t*)w.fronts[nf].p;
    ++nf;
    return r;
  };
  auto update = [&](const uint32_t* N, int64_t* cnt_out) -> int {
    if (n > 0) {
      auto* so = (uint32_t*)w.S.p;
      auto* fz = (uint32_t*)w.fnz.p;
      auto* po = (uint32_t*)w.part_or.p;
      auto* pc = (int64_t*)w.part_cnt.p;
      if (upd_v == 4)
        k_bfs_update<4><<<(unsigned)nblk, 256, 0, st>>>(n, wp, N, so, fz, po, pc);
      else if (upd_v == 2)
        k_bfs_update<2><<<(unsigned)nblk, 256, 0, st>>>(n, wp, N, so, fz, po, pc);
      else
        k_bfs_update<1><<<(unsigned)nblk, 256, 0, st>>>(n, wp, N, so, fz, po, pc);
    }
    k_bfs_reduce<<<1, 1024, 0, st>>>(n > 0 ? nblk : 0, wp, (const uint32_t*)w.part_or.p,
                                     (const int64_t*)w.part_cnt.p, (uint32_t*)w.active.p, (int64_t*)w.count.p);
    TSS_CHECK_LAUNCH();
    TSS_HIP(hipMemcpyAsync(w.host_count, w.count.p, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TSS_HIP(hipStreamSynchronize(st));
    *cnt_out = *w.host_count;
    return TSSPGEMM_OK;
  };

  // N_0 = one-hot sources; S = N_0
  uint32_t* f0 = nullptr;
  if ((rc = new_front(&f0))) return rc;
  if ((rc = launch_zero_bytes(f0, (size_t)n * wp * 4, st)) || (rc = launch_zero_bytes(w.S.p, (size_t)n * wp * 4, st)) ||
      (rc = launch_zero_bytes(w.count.p, 16, st)))
    return rc;
  k_bfs_seed<<<grid_for(d, 256), 256, 0, st>>>(sources, d, n, wp, f0, (int64_t*)w.count.p + 1);
  TSS_CHECK_LAUNCH();
  int64_t cnt = 0;
  if ((rc = update(f0, &cnt))) return rc;
  if (w.host_count[1]) {
    set_error("msbfs: a source vertex is outside [0, n)");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  int32_t it = 0;
  while (cnt > 0) {
    ++it;
    uint32_t* nt = nullptr;
    if ((rc = new_front(&nt))) return rc;
    pr.bbits = (const uint32_t*)w.fronts[nf - 2].p;
    pr.cbits = nt;
    SymParams sp{};
    sp.pr = pr;
    sp.items = (const Item*)p.sym_items.p;
    sp.ctr = ctr;
    sp.mask = (const uint32_t*)w.S.p;
    sp.active = (const uint32_t*)w.active.p;
    sp.fnz = (const uint32_t*)w.fnz.p;
    sp.early_exit = true;
    sp.light_max = kSlotRowMaxBfs;
    if ((rc = launch_sym_split_zero(pr, sp.items, ctr, sym_cap, st)) || (rc = launch_symbolic(sp, sym_cap, st)) ||
        (rc = launch_sym_split_mask(pr, sp.items, sp.mask, ctr, sym_cap, st)))
      return rc;
    if ((rc = update(nt, &cnt))) return rc;
    if (frontier_nnz && it <= capacity) frontier_nnz[it - 1] = cnt;
  }
  // levels from the kept frontiers N_0 .. N_T (the last one is empty)
  const int32_t nfront = (int32_t)nf - 1;
  std::vector<const uint32_t*> fp(nfront);
  for (int t = 0; t < nfront; ++t) fp[t] = (const uint32_t*)w.fronts[t].p;
  if ((rc = w.fronts_dev.ensure(sizeof(void*) * (nfront + 1)))) return rc;
  TSS_HIP(hipMemcpyAsync(w.fronts_dev.p, fp.data(), sizeof(void*) * nfront, hipMemcpyHostToDevice, st));
  if (nfront <= 32 && (d & 31) == 0 && ((uintptr_t)levels & 15) == 0) {
    const int64_t words = n * (d >> 5);
    if (words > 0) {
      k_bfs_levels_words<<<(int)std::min<int64_t>((words + 255) / 256, 2048), 256, 0, st>>>(
          n, d, wp, nfront, (const uint32_t* const*)w.fronts_dev.p, levels);
      TSS_CHECK_LAUNCH();
    }
  } else {
    const int64_t waves = n * ((d + 255) / 256);
    if (waves > 0) {
      k_bfs_levels<<<(int)std::min<int64_t>((waves + 3) / 4, 8192), 256, 0, st>>>(
          n, d, wp, nfront, (const uint32_t* const*)w.fronts_dev.p, levels);
      TSS_CHECK_LAUNCH();
    }
  }
  TSS_HIP(hipStreamSynchronize(st));
  *iterations = it;
  return TSSPGEMM_OK;
}

}  // namespace tss

extern "C" int tsspgemm_msbfs(const tsspgemm_csr* A, const int32_t* sources, int32_t d, int32_t* levels,
                              int32_t* iterations, int64_t* frontier_nnz, int32_t capacity, void* stream) {
  try {
    return tss::run_msbfs(A, sources, d, levels, iterations, frontier_nnz, capacity, (hipStream_t)stream);
  } catch (...) {
    tss::set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}
