// Seeded synthetic input generators for TS-SpGEMM workloads.
//
// This file holds NO arithmetic of the multiply itself: it only draws random
// matrices (Erdos-Renyi and R-MAT graphs, tall-and-skinny B patterns, BFS
// sources, loss weights) in CSR form with sorted, unique column indices.
// Both the CPU oracle and the GPU path consume what it produces.
//
// Randomness: every draw is the i-th output of a SplitMix64 sequence
// (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014; finaliser constants as published by Vigna), evaluated in
// counter form  out(key, i) = mix64(key + (i + 1) * GAMMA), so results do not
// depend on the number of OpenMP threads.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ULL;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
inline uint64_t stream_key(uint64_t seed, uint64_t stream) { return mix64(mix64(seed + GAMMA) ^ (stream * GAMMA)); }
inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GAMMA); }
// uniform double in [0,1)
inline double unit(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
// uniform integer in [0, n)  (multiply-shift)
inline uint64_t below(uint64_t r, uint64_t n) { return (uint64_t)(((unsigned __int128)r * n) >> 64); }
// U(0,1] on the FP32 grid: (m+1) * 2^-24, never 0, exactly representable
inline float unit_f32(uint64_t r) { return (float)((double)((r >> 40) + 1) * 0x1.0p-24); }
// N(0,1) by Box-Muller from two consecutive draws
inline float normal_f32(uint64_t key, uint64_t i) {
  double u1 = ((double)(draw(key, 2 * i) >> 11) + 1.0) * 0x1.0p-53;  // (0,1]
  double u2 = unit(draw(key, 2 * i + 1));
  return (float)(std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
}

// Streams (distinct purposes never share a key).
enum : uint64_t {
  S_ER_COL = 1, S_RMAT = 2, S_AVAL = 3, S_BPAT = 4, S_BVAL = 5, S_BLEN = 6,
  S_BCOL = 7, S_SRC = 8, S_W = 9, S_AVALN = 10, S_NEG = 11, S_ZCOL = 12, S_ZVAL = 13,
};

// Build a CSR with sorted unique columns from per-row unsorted column lists.
// rows[i] holds row i's columns. Returns nnz; fills rp (n+1) and ci.
struct Csr {
  std::vector<int32_t> rp, ci;
};

void sort_dedup_rows(int64_t n, std::vector<int64_t>& rp64, std::vector<int32_t>& cols, Csr& out) {
  std::vector<int32_t> len(n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    int32_t* b = cols.data() + rp64[i];
    int32_t* e = cols.data() + rp64[i + 1];
    std::sort(b, e);
    len[i] = (int32_t)(std::unique(b, e) - b);
  }
  out.rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) out.rp[i + 1] = out.rp[i] + len[i];
  out.ci.resize(out.rp[n]);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i)
    std::memcpy(out.ci.data() + out.rp[i], cols.data() + rp64[i], sizeof(int32_t) * len[i]);
}

// Symmetrise an edge list (drop self-loops), dedup, CSR.
void edges_to_sym_csr(int64_t n, const std::vector<int32_t>& u, const std::vector<int32_t>& v, Csr& out) {
  int64_t m = (int64_t)u.size();
  std::vector<std::atomic<int64_t>> deg(n);
  for (int64_t i = 0; i < n; ++i) deg[i].store(0, std::memory_order_relaxed);
#pragma omp parallel for
  for (int64_t e = 0; e < m; ++e) {
    if (u[e] == v[e]) continue;
    deg[u[e]].fetch_add(1, std::memory_order_relaxed);
    deg[v[e]].fetch_add(1, std::memory_order_relaxed);
  }
  std::vector<int64_t> rp64(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) rp64[i + 1] = rp64[i] + deg[i].load(std::memory_order_relaxed);
  std::vector<int32_t> cols(rp64[n]);
  std::vector<std::atomic<int64_t>> pos(n);
  for (int64_t i = 0; i < n; ++i) pos[i].store(rp64[i], std::memory_order_relaxed);
#pragma omp parallel for
  for (int64_t e = 0; e < m; ++e) {
    if (u[e] == v[e]) continue;
    cols[pos[u[e]].fetch_add(1, std::memory_order_relaxed)] = v[e];
    cols[pos[v[e]].fetch_add(1, std::memory_order_relaxed)] = u[e];
  }
  sort_dedup_rows(n, rp64, cols, out);
}

void rmat_edge(uint64_t key, uint64_t e, int scale, double a, double b, double c, int32_t& u, int32_t& v) {
  uint32_t r = 0, s = 0;
  for (int l = 0; l < scale; ++l) {
    double x = unit(draw(key, e * 64 + (uint64_t)l));
    uint32_t bit = 1u << (scale - 1 - l);
    if (x < a) {
    } else if (x < a + b) {
      s |= bit;
    } else if (x < a + b + c) {
      r |= bit;
    } else {
      r |= bit;
      s |= bit;
    }
  }
  u = (int32_t)r;
  v = (int32_t)s;
}

// Result handle passed back to Python: owns the arrays until freed.
struct Result {
  int64_t n = 0, ncols = 0;
  std::vector<int32_t> rp, ci;
  std::vector<float> val;
};

}  // namespace

extern "C" {

uint64_t synth_draw(uint64_t seed, uint64_t stream, uint64_t i) { return draw(stream_key(seed, stream), i); }
double synth_unit(uint64_t seed, uint64_t stream, uint64_t i) { return unit(draw(stream_key(seed, stream), i)); }

void* synth_er(int64_t n, int32_t draws, uint64_t seed) {
  uint64_t key = stream_key(seed, S_ER_COL);
  std::vector<int64_t> rp64(n + 1);
  for (int64_t i = 0; i <= n; ++i) rp64[i] = i * draws;
  std::vector<int32_t> cols((size_t)n * draws);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i)
    for (int t = 0; t < draws; ++t) cols[i * draws + t] = (int32_t)below(draw(key, (uint64_t)(i * draws + t)), (uint64_t)n);
  Result* r = new Result;
  Csr c;
  sort_dedup_rows(n, rp64, cols, c);
  r->n = n;
  r->ncols = n;
  r->rp.swap(c.rp);
  r->ci.swap(c.ci);
  return r;
}

// R-MAT graph on n vertices (n <= 2^scale). When n < 2^scale, edges with an
// endpoint >= n are rejected until `nedges` are accepted (in counter order).
// The result is symmetrised, without self-loops, with duplicates merged.
void* synth_rmat(int32_t scale, int64_t n, int64_t nedges, double a, double b, double c, uint64_t seed) {
  uint64_t key = stream_key(seed, S_RMAT);
  std::vector<int32_t> u, v;
  if (n == ((int64_t)1 << scale)) {
    u.resize(nedges);
    v.resize(nedges);
#pragma omp parallel for
    for (int64_t e = 0; e < nedges; ++e) rmat_edge(key, (uint64_t)e, scale, a, b, c, u[e], v[e]);
  } else {
    const int64_t chunk = 1 << 20;
    u.reserve(nedges);
    v.reserve(nedges);
    std::vector<int32_t> cu(chunk), cv(chunk);
    int64_t base = 0;
    while ((int64_t)u.size() < nedges) {
#pragma omp parallel for
      for (int64_t e = 0; e < chunk; ++e) rmat_edge(key, (uint64_t)(base + e), scale, a, b, c, cu[e], cv[e]);
      for (int64_t e = 0; e < chunk && (int64_t)u.size() < nedges; ++e)
        if (cu[e] < n && cv[e] < n) {
          u.push_back(cu[e]);
          v.push_back(cv[e]);
        }
      base += chunk;
    }
  }
  Result* r = new Result;
  Csr cs;
  edges_to_sym_csr(n, u, v, cs);
  r->n = n;
  r->ncols = n;
  r->rp.swap(cs.rp);
  r->ci.swap(cs.ci);
  return r;
}

// Tall-and-skinny n x d pattern, each entry present with probability p.
void* synth_b_bernoulli(int64_t n, int32_t d, double p, uint64_t seed) {
  uint64_t key = stream_key(seed, S_BPAT);
  std::vector<int32_t> len(n);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    int32_t k = 0;
    for (int32_t j = 0; j < d; ++j) k += unit(draw(key, (uint64_t)(i * d + j))) < p;
    len[i] = k;
  }
  Result* r = new Result;
  r->n = n;
  r->ncols = d;
  r->rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) r->rp[i + 1] = r->rp[i] + len[i];
  r->ci.resize(r->rp[n]);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    int32_t* o = r->ci.data() + r->rp[i];
    for (int32_t j = 0; j < d; ++j)
      if (unit(draw(key, (uint64_t)(i * d + j))) < p) *o++ = j;
  }
  return r;
}

// Tall-and-skinny n x d pattern with Poisson(lam) entries per row (inversion,
// truncated at d) at uniformly random distinct columns (Floyd's algorithm).
void* synth_b_poisson(int64_t n, int32_t d, double lam, uint64_t seed) {
  uint64_t klen = stream_key(seed, S_BLEN), kcol = stream_key(seed, S_BCOL);
  std::vector<int32_t> len(n);
  const double p0 = std::exp(-lam);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    double x = unit(draw(klen, (uint64_t)i));
    int32_t k = 0;
    double pk = p0, cdf = p0;
    while (x >= cdf && k < d) {
      ++k;
      pk *= lam / k;
      cdf += pk;
      if (pk == 0.0) break;
    }
    len[i] = std::min(k, d);
  }
  Result* r = new Result;
  r->n = n;
  r->ncols = d;
  r->rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) r->rp[i + 1] = r->rp[i] + len[i];
  r->ci.resize(r->rp[n]);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    int32_t L = len[i];
    int32_t* o = r->ci.data() + r->rp[i];
    int32_t cnt = 0;
    for (int32_t j = d - L; j < d; ++j) {  // Floyd: pick L distinct of [0,d)
      int32_t t = (int32_t)below(draw(kcol, (uint64_t)(i * d + j)), (uint64_t)(j + 1));
      bool seen = false;
      for (int32_t q = 0; q < cnt; ++q) seen |= (o[q] == t);
      o[cnt++] = seen ? j : t;
    }
    std::sort(o, o + L);
  }
  return r;
}

int64_t synth_n(void* h) { return ((Result*)h)->n; }
int64_t synth_nnz(void* h) { return (int64_t)((Result*)h)->ci.size(); }
void synth_copy(void* h, int32_t* rp, int32_t* ci) {
  Result* r = (Result*)h;
  std::memcpy(rp, r->rp.data(), sizeof(int32_t) * r->rp.size());
  std::memcpy(ci, r->ci.data(), sizeof(int32_t) * r->ci.size());
}
void synth_free(void* h) { delete (Result*)h; }

// Values for stored entries, keyed by the entry's (row, col) position
// row * ncols + col, so a value does not depend on which other entries exist.
// kind 0: U(0,1] on the FP32 grid;  kind 1: N(0,1);  kind 2: integers in
// [-range, range] (as float, exact).
void synth_values(const int32_t* rp, const int32_t* ci, int64_t nrows, int64_t ncols, int32_t kind, int32_t range,
                  uint64_t seed, uint64_t stream, float* out) {
  uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < nrows; ++i)
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
      uint64_t idx = (uint64_t)(i * ncols + ci[p]);
      float x;
      if (kind == 0)
        x = unit_f32(draw(key, idx));
      else if (kind == 1)
        x = normal_f32(key, idx);
      else
        x = (float)((int64_t)below(draw(key, idx), (uint64_t)(2 * range + 1)) - range);
      out[p] = x;
    }
}

// d distinct sources drawn uniformly among vertices with at least one stored
// entry in their row (non-isolated). Returns the number found (< d only if
// fewer non-isolated vertices exist).
int32_t synth_sources(const int32_t* rp, int64_t n, int32_t d, uint64_t seed, int32_t* out) {
  uint64_t key = stream_key(seed, S_SRC);
  int64_t nonisolated = 0;
  for (int64_t i = 0; i < n; ++i) nonisolated += rp[i + 1] > rp[i];
  int32_t want = (int32_t)std::min<int64_t>(d, nonisolated);
  std::vector<char> taken(n, 0);
  int32_t got = 0;
  for (uint64_t t = 0; got < want; ++t) {
    int64_t v = (int64_t)below(draw(key, t), (uint64_t)n);
    if (rp[v + 1] > rp[v] && !taken[v]) {
      taken[v] = 1;
      out[got++] = (int32_t)v;
    }
  }
  return got;
}

// Negative samples for a graph embedding: for each vertex i, `ns` distinct
// vertices drawn uniformly among those that are neither i nor a neighbour of i
// (rejection in counter order: draw t of row i is draw(key, i * 4096 + t),
// t < 4096, so a row with almost no non-neighbours may get fewer). Returns
// the samples as a CSR pattern with sorted columns.
void* synth_negatives(const int32_t* rp, const int32_t* ci, int64_t n, int32_t ns, uint64_t seed) {
  uint64_t key = stream_key(seed, S_NEG);
  std::vector<int32_t> len(n);
  std::vector<int32_t> cols((size_t)n * ns);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    int32_t* o = cols.data() + (size_t)i * ns;
    int32_t got = 0;
    for (uint64_t t = 0; t < 4096 && got < ns; ++t) {
      const int32_t v = (int32_t)below(draw(key, (uint64_t)i * 4096 + t), (uint64_t)n);
      if (v == i || std::binary_search(ci + rp[i], ci + rp[i + 1], v)) continue;
      bool seen = false;
      for (int32_t q = 0; q < got; ++q) seen |= (o[q] == v);
      if (!seen) o[got++] = v;
    }
    std::sort(o, o + got);
    len[i] = got;
  }
  Result* r = new Result;
  r->n = n;
  r->ncols = n;
  r->rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) r->rp[i + 1] = r->rp[i] + len[i];
  r->ci.resize(r->rp[n]);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i)
    std::copy(cols.data() + (size_t)i * ns, cols.data() + (size_t)i * ns + len[i], r->ci.data() + r->rp[i]);
  return r;
}

// Initial sparse embedding: every row of the n x d matrix holds exactly k
// entries at distinct uniform columns (Floyd's algorithm), sorted, stored at
// row i * k; values N(0,1) scaled by 1/sqrt(k) (rounded once to FP32), keyed
// by (row, column).
void synth_embed_init(int64_t n, int32_t d, int32_t k, uint64_t seed, int32_t* ci, float* val) {
  uint64_t kcol = stream_key(seed, S_ZCOL), kval = stream_key(seed, S_ZVAL);
  const double scale = 1.0 / std::sqrt((double)k);
#pragma omp parallel for
  for (int64_t i = 0; i < n; ++i) {
    int32_t* o = ci + i * k;
    int32_t cnt = 0;
    for (int32_t j = d - k; j < d; ++j) {
      int32_t t = (int32_t)below(draw(kcol, (uint64_t)(i * d + j)), (uint64_t)(j + 1));
      bool seen = false;
      for (int32_t q = 0; q < cnt; ++q) seen |= (o[q] == t);
      o[cnt++] = seen ? j : t;
    }
    std::sort(o, o + k);
    for (int32_t q = 0; q < k; ++q)
      val[i * k + q] = (float)((double)normal_f32(kval, (uint64_t)(i * d + o[q])) * scale);
  }
}

}  // extern "C"
