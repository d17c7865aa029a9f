// CPU ORACLE for TS-SpGEMM -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, obviously-correct reference implementations of what the GPU
// library computes. Only the test-suite, the smoke check and the benchmark's
// CPU-baseline leg may load this. It shares no code, header, table or helper
// with the GPU library, and never includes anything from it.
//
// Definitions followed (paper: "Distributed-Memory Parallel Algorithms for
// Sparse Matrix and Sparse Tall-and-Skinny Matrix Multiplication", SC'24):
//  * Sec. II-A: C = A B with A n x n, B n x d; any semiring; "flops" is the
//    number of multiplications needed to form A B.
//  * Sec. III-A, Eq. (1): row-wise Gustavson, C(r,:) = sum over c with
//    A(r,c) != 0 of A(r,c) * B(c,:).
//  * Sec. IV-A, Algorithm 3: multi-source BFS over the (AND, OR) semiring:
//    N = A F, F = N \ S, S = S v N, repeat while nnz(F) > 0.
//  * Sec. IV-B: sparse force-directed embedding. Neighbours pull and
//    negative samples push; the forces are a TS-SpGEMM of the signed graph
//    with the embedding, followed by an SGD step and re-sparsification of
//    each updated row to its largest entries; rows are updated in minibatches.
//  * Sec. III-B / III-C, Algorithm 2: A is processed tile by tile (a tile
//    takes a range of A's columns); the partial products of the tiles are
//    merged into C. The merge of partial outputs is their sum, row by row.
//  * Backward of L = sum(C o W) (no counterpart in the paper; definitions of
//    the derivative of a bilinear form): dL/dA(i,k) = sum_j G(i,j) B(k,j) on
//    pat(A), dL/dB(k,j) = sum_i A(i,k) G(i,j) on pat(B), G = W on pat(C).
//
// Readings taken where the paper is silent:
//  * C's pattern is the structural product: every column touched by some
//    A(i,k) B(k,j) is stored, even when its numeric sum is zero.
//  * Columns within a row are emitted in ascending order, without duplicates.
//  * Floating point is FP64 throughout. FP32 inputs convert exactly and every
//    FP32 x FP32 product is exact in FP64; sums run in ascending k order.
//  * The (AND, OR) semiring of the paper is written (multiply, add), so the
//    multiply is AND and the add is OR.
//  * Complement mask: entries whose column is stored in the mask row are
//    dropped from the output row.
//  * Embedding forces (the paper names Force2Vec without its formula): the
//    sigmoid model of negative sampling. For a stored entry (i, j) with sign
//    a of the signed graph, s = z_i . z_j, sig = 1 / (1 + exp(-s)), weight
//    w = 1 - sig if a > 0, -sig if a < 0, 0 if a = 0; F_i = sum_j w z_j is the
//    gradient in z_i of sum log sig(+-z_i . z_j). Update u = z_i + lr F_i in
//    FP64, rounded once to FP32. "Keeping the highest valued entries" is read
//    as the k largest |u| (ties: lower column), so every row keeps exactly k
//    entries (zeros included when fewer are nonzero), sorted by column.
//    Within a minibatch every row reads the embedding as it was at the start
//    of the minibatch; minibatches run in row order, each seeing the ones
//    before it.
//  * BFS levels: level 0 at the sources, t at the iteration that first adds
//    the vertex to S, -1 if never reached. "Neighbours" follow A F: vertex i
//    is reached from k when A(i,k) != 0.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <thread>
#include <utility>
#include <vector>

namespace {

struct Rows {  // an output with one row per selected input row
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> val;
};

// Run fn(t) for t in [0, count) split in contiguous static chunks over
// `threads` std::threads. The arithmetic of each t does not depend on the split.
template <class F>
void for_rows(int64_t count, int threads, F fn) {
  if (threads <= 1 || count < 2) {
    for (int64_t t = 0; t < count; ++t) fn(t);
    return;
  }
  std::vector<std::thread> pool;
  int64_t per = (count + threads - 1) / threads;
  for (int w = 0; w < threads; ++w) {
    int64_t lo = w * per, hi = lo + per < count ? lo + per : count;
    if (lo >= hi) break;
    pool.emplace_back([=] {
      for (int64_t t = lo; t < hi; ++t) fn(t);
    });
  }
  for (auto& th : pool) th.join();
}

Rows* gather_rows(std::vector<std::map<int32_t, double>>& maps) {
  Rows* r = new Rows;
  r->rp.assign(maps.size() + 1, 0);
  for (size_t t = 0; t < maps.size(); ++t) r->rp[t + 1] = r->rp[t] + (int64_t)maps[t].size();
  r->ci.resize(r->rp.back());
  r->val.resize(r->rp.back());
  for (size_t t = 0; t < maps.size(); ++t) {
    int64_t o = r->rp[t];
    for (auto& kv : maps[t]) {  // std::map iterates keys in ascending order
      r->ci[o] = kv.first;
      r->val[o] = kv.second;
      ++o;
    }
  }
  return r;
}

}  // namespace

extern "C" {

// flops per row (Sec. II-A): number of multiplications A(i,k) B(k,j) in row i.
void oracle_row_flops(int64_t n, const int32_t* arp, const int32_t* aci, const int32_t* brp, int64_t* flops) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t f = 0;
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p) f += brp[aci[p] + 1] - brp[aci[p]];
    flops[i] = f;
  }
}

// Plus-times over FP64 (Eq. 1, row-wise Gustavson with an ordered map per
// row). rows == nullptr selects all n rows; otherwise the nsel listed rows.
void* oracle_spgemm_f64(int64_t n, const int32_t* arp, const int32_t* aci, const double* aval, const int32_t* brp,
                        const int32_t* bci, const double* bval, const int32_t* rows, int64_t nsel, int threads) {
  int64_t count = rows ? nsel : n;
  std::vector<std::map<int32_t, double>> maps(count);
  for_rows(count, threads, [&](int64_t t) {
    int64_t i = rows ? rows[t] : t;
    std::map<int32_t, double>& acc = maps[t];
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
      int32_t k = aci[p];
      double a = aval[p];
      for (int32_t q = brp[k]; q < brp[k + 1]; ++q) acc[bci[q]] += a * bval[q];
    }
  });
  return gather_rows(maps);
}

// Plus-times over integers: int64 accumulation (callers keep |values| small
// enough that every sum fits int32; the Python wrapper checks that).
void* oracle_spgemm_i64(int64_t n, const int32_t* arp, const int32_t* aci, const int64_t* aval, const int32_t* brp,
                        const int32_t* bci, const int64_t* bval, const int32_t* rows, int64_t nsel, int threads) {
  int64_t count = rows ? nsel : n;
  std::vector<std::map<int32_t, int64_t>> maps(count);
  for_rows(count, threads, [&](int64_t t) {
    int64_t i = rows ? rows[t] : t;
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
      int32_t k = aci[p];
      for (int32_t q = brp[k]; q < brp[k + 1]; ++q) maps[t][bci[q]] += aval[p] * bval[q];
    }
  });
  Rows* r = new Rows;
  r->rp.assign(count + 1, 0);
  for (int64_t t = 0; t < count; ++t) r->rp[t + 1] = r->rp[t] + (int64_t)maps[t].size();
  r->ci.resize(r->rp.back());
  r->val.resize(r->rp.back());
  for (int64_t t = 0; t < count; ++t) {
    int64_t o = r->rp[t];
    for (auto& kv : maps[t]) {
      r->ci[o] = kv.first;
      r->val[o] = (double)kv.second;  // exact: |sum| < 2^53 for every test input
      ++o;
    }
  }
  return r;
}

// (AND, OR) semiring with optional complement mask: row i of the output is
// the union of pat(B_k) over k in pat(A_i), minus the columns of mask row i.
void* oracle_spgemm_bool(int64_t n, const int32_t* arp, const int32_t* aci, const int32_t* brp, const int32_t* bci,
                         const int32_t* mrp, const int32_t* mci, const int32_t* rows, int64_t nsel, int threads) {
  int64_t count = rows ? nsel : n;
  std::vector<std::set<int32_t>> sets(count);
  for_rows(count, threads, [&](int64_t t) {
    int64_t i = rows ? rows[t] : t;
    std::set<int32_t>& s = sets[t];
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p)
      for (int32_t q = brp[aci[p]]; q < brp[aci[p] + 1]; ++q) s.insert(bci[q]);
    if (mrp)
      for (int32_t q = mrp[i]; q < mrp[i + 1]; ++q) s.erase(mci[q]);
  });
  Rows* r = new Rows;
  r->rp.assign(count + 1, 0);
  for (int64_t t = 0; t < count; ++t) r->rp[t + 1] = r->rp[t] + (int64_t)sets[t].size();
  r->ci.resize(r->rp.back());
  for (int64_t t = 0; t < count; ++t) {
    int64_t o = r->rp[t];
    for (int32_t j : sets[t]) r->ci[o++] = j;
  }
  return r;
}

int64_t oracle_res_rows(void* h) { return (int64_t)((Rows*)h)->rp.size() - 1; }
int64_t oracle_res_nnz(void* h) { return ((Rows*)h)->rp.back(); }
void oracle_res_copy(void* h, int64_t* rp, int32_t* ci, double* val) {
  Rows* r = (Rows*)h;
  std::memcpy(rp, r->rp.data(), sizeof(int64_t) * r->rp.size());
  std::memcpy(ci, r->ci.data(), sizeof(int32_t) * r->ci.size());
  if (val && !r->val.empty()) std::memcpy(val, r->val.data(), sizeof(double) * r->val.size());
}
void oracle_res_free(void* h) { delete (Rows*)h; }

// Transpose of an n x m CSR by a row-order walk: entry (i,k) is appended to
// row k of the transpose, so each transposed row lists i ascending.
// perm[q] is the position in A of the entry stored at q in the transpose.
void oracle_transpose(int64_t n, int64_t m, const int32_t* arp, const int32_t* aci, int32_t* trp, int32_t* tci,
                      int32_t* perm) {
  std::vector<std::vector<std::pair<int32_t, int32_t>>> cols(m);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p) cols[aci[p]].push_back({(int32_t)i, p});
  trp[0] = 0;
  for (int64_t k = 0; k < m; ++k) {
    trp[k + 1] = trp[k] + (int32_t)cols[k].size();
    int32_t o = trp[k];
    for (auto& e : cols[k]) {
      tci[o] = e.first;
      perm[o] = e.second;
      ++o;
    }
  }
}

// Multi-source BFS by Algorithm 3 with ordered sets: F, S, N as per-row sets
// of source columns. levels is n x d (row-major), -1 where unreachable.
// Returns the number of iterations with a non-empty frontier.
// frontier_flops (may be null, capacity 4096): per iteration, the
// multiplications of that iteration's product A F (Sec. II-A: one per pair of
// a stored A(i,k) and a stored F(k,s)), counted before F is replaced.
int32_t oracle_msbfs(int64_t n, const int32_t* arp, const int32_t* aci, const int32_t* src, int32_t d,
                     int32_t* levels, int64_t* frontier_nnz /* per iteration, may be null, capacity 4096 */,
                     int64_t* frontier_flops) {
  for (int64_t x = 0; x < n * (int64_t)d; ++x) levels[x] = -1;
  std::vector<std::set<int32_t>> F(n), S(n);
  for (int32_t j = 0; j < d; ++j) {
    F[src[j]].insert(j);
    S[src[j]].insert(j);
    levels[(int64_t)src[j] * d + j] = 0;
  }
  int32_t iter = 0;
  auto nnzF = [&] {
    int64_t s = 0;
    for (auto& r : F) s += (int64_t)r.size();
    return s;
  };
  while (nnzF() > 0) {
    ++iter;
    std::vector<std::set<int32_t>> N(n);
    int64_t mults = 0;
    for (int64_t i = 0; i < n; ++i)  // N = A F over (AND, OR)
      for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
        N[i].insert(F[aci[p]].begin(), F[aci[p]].end());
        mults += (int64_t)F[aci[p]].size();
      }
    if (frontier_flops && iter <= 4096) frontier_flops[iter - 1] = mults;
    for (int64_t i = 0; i < n; ++i) {
      std::set<int32_t> next;  // F = N \ S
      for (int32_t j : N[i])
        if (!S[i].count(j)) next.insert(j);
      F[i].swap(next);
      for (int32_t j : N[i]) S[i].insert(j);  // S = S v N
      for (int32_t j : F[i]) levels[i * (int64_t)d + j] = iter;
    }
    if (frontier_nnz && iter <= 4096) frontier_nnz[iter - 1] = nnzF();
  }
  return iter;
}

// Independent check of the BFS: one plain queue BFS per source. Vertex i is
// reached from k when A(i,k) != 0, so the out-list of k is column k of A.
void oracle_bfs_queue(int64_t n, const int32_t* arp, const int32_t* aci, const int32_t* src, int32_t d,
                      int32_t* levels, int threads) {
  std::vector<std::vector<int32_t>> out(n);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p) out[aci[p]].push_back((int32_t)i);
  for (int64_t x = 0; x < n * (int64_t)d; ++x) levels[x] = -1;
  for_rows(d, threads, [&](int64_t j) {
    std::vector<int32_t> lev(n, -1);
    std::deque<int32_t> q;
    lev[src[j]] = 0;
    q.push_back(src[j]);
    while (!q.empty()) {
      int32_t v = q.front();
      q.pop_front();
      for (int32_t u : out[v])
        if (lev[u] < 0) {
          lev[u] = lev[v] + 1;
          q.push_back(u);
        }
    }
    for (int64_t i = 0; i < n; ++i) levels[i * (int64_t)d + j] = lev[i];
  });
}

// dL/dA(i,k) = sum over j in pat(B_k) of G(i,j) B(k,j), for (i,k) in pat(A).
// G is given on pat(C) (C = A B); every needed G(i,j) lies there. Returns 0,
// or -1 if some needed G entry is missing from C's pattern.
int oracle_grad_a(int64_t n, const int32_t* arp, const int32_t* aci, const int32_t* brp, const int32_t* bci,
                  const double* bval, const int32_t* crp, const int32_t* cci, const double* g, double* grad_a) {
  int bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    std::map<int32_t, double> grow;
    for (int32_t q = crp[i]; q < crp[i + 1]; ++q) grow[cci[q]] = g[q];
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
      int32_t k = aci[p];
      double s = 0.0;
      for (int32_t q = brp[k]; q < brp[k + 1]; ++q) {
        auto it = grow.find(bci[q]);
        if (it == grow.end()) {
          bad = 1;
          continue;
        }
        s += it->second * bval[q];
      }
      grad_a[p] = s;
    }
  }
  return bad ? -1 : 0;
}

// dL/dB(k,j) = sum over i with A(i,k) != 0 of A(i,k) G(i,j), for (k,j) in
// pat(B), accumulated over A's rows in order into an ordered map.
int oracle_grad_b(int64_t n, const int32_t* arp, const int32_t* aci, const double* aval, const int32_t* brp,
                  const int32_t* bci, const int32_t* crp, const int32_t* cci, const double* g, double* grad_b) {
  std::map<std::pair<int32_t, int32_t>, double> acc;
  int bad = 0;
  for (int64_t i = 0; i < n; ++i) {
    std::map<int32_t, double> grow;
    for (int32_t q = crp[i]; q < crp[i + 1]; ++q) grow[cci[q]] = g[q];
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
      int32_t k = aci[p];
      for (int32_t q = brp[k]; q < brp[k + 1]; ++q) {
        auto it = grow.find(bci[q]);
        if (it == grow.end()) {
          bad = 1;
          continue;
        }
        acc[{k, bci[q]}] += aval[p] * it->second;
      }
    }
  }
  for (int64_t k = 0; k < n; ++k)
    for (int32_t q = brp[k]; q < brp[k + 1]; ++q) {
      auto it = acc.find({(int32_t)k, bci[q]});
      grad_b[q] = it == acc.end() ? 0.0 : it->second;
    }
  return bad ? -1 : 0;
}

// Sampled forms for full-size checks: dL/dA on the rows listed in `rows`
// (output laid out as those rows' A entries, concatenated), and dL/dB on the
// B rows listed in `krows` (output laid out as those rows' B entries).
int oracle_grad_a_rows(const int32_t* arp, const int32_t* aci, const int32_t* brp, const int32_t* bci,
                       const double* bval, const int32_t* crp, const int32_t* cci, const double* g,
                       const int32_t* rows, int64_t nsel, double* out) {
  int bad = 0;
  int64_t o = 0;
  for (int64_t t = 0; t < nsel; ++t) {
    int32_t i = rows[t];
    std::map<int32_t, double> grow;
    for (int32_t q = crp[i]; q < crp[i + 1]; ++q) grow[cci[q]] = g[q];
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
      int32_t k = aci[p];
      double s = 0.0;
      for (int32_t q = brp[k]; q < brp[k + 1]; ++q) {
        auto it = grow.find(bci[q]);
        if (it == grow.end()) {
          bad = 1;
          continue;
        }
        s += it->second * bval[q];
      }
      out[o++] = s;
    }
  }
  return bad ? -1 : 0;
}

int oracle_grad_b_rows(int64_t n, const int32_t* arp, const int32_t* aci, const double* aval, const int32_t* brp,
                       const int32_t* bci, const int32_t* crp, const int32_t* cci, const double* g,
                       const int32_t* krows, int64_t nsel, double* out) {
  std::map<int32_t, int64_t> slot;  // selected k -> index in krows
  for (int64_t t = 0; t < nsel; ++t) slot[krows[t]] = t;
  std::vector<std::vector<std::pair<int32_t, double>>> colk(nsel);  // (i, A(i,k)), i ascending
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
      auto it = slot.find(aci[p]);
      if (it != slot.end()) colk[it->second].push_back({(int32_t)i, aval[p]});
    }
  int bad = 0;
  int64_t o = 0;
  for (int64_t t = 0; t < nsel; ++t) {
    int32_t k = krows[t];
    std::map<int32_t, double> acc;
    for (auto& e : colk[t]) {
      int32_t i = e.first;
      std::map<int32_t, double> grow;
      for (int32_t q = crp[i]; q < crp[i + 1]; ++q) grow[cci[q]] = g[q];
      for (int32_t q = brp[k]; q < brp[k + 1]; ++q) {
        auto it = grow.find(bci[q]);
        if (it == grow.end()) {
          bad = 1;
          continue;
        }
        acc[bci[q]] += e.second * it->second;
      }
    }
    for (int32_t q = brp[k]; q < brp[k + 1]; ++q) out[o++] = acc.count(bci[q]) ? acc[bci[q]] : 0.0;
  }
  return bad ? -1 : 0;
}

// ---------------------------------------------------------------- embedding

// Force on row i (Sec. IV-B, sigmoid negative-sampling reading): F = sum over
// the stored entries (i, j, a) of the signed graph, in column order, of
// w(a, z_i . z_j) z_j. z rows are k entries each, stored at row * k.
void oracle_embed_force(const int32_t* arp, const int32_t* aci, const float* aval, int64_t d, int64_t k,
                        const int32_t* zci, const float* zval, int64_t i, double* F) {
  std::vector<double> zi(d, 0.0);
  for (int64_t t = 0; t < k; ++t) zi[zci[i * k + t]] = zval[i * k + t];
  for (int64_t c = 0; c < d; ++c) F[c] = 0.0;
  for (int32_t p = arp[i]; p < arp[i + 1]; ++p) {
    const int64_t j = aci[p];
    const double a = aval[p];
    double s = 0.0;
    for (int64_t t = 0; t < k; ++t) s += zi[zci[j * k + t]] * (double)zval[j * k + t];
    const double sig = 1.0 / (1.0 + std::exp(-s));
    const double w = a > 0 ? 1.0 - sig : (a < 0 ? -sig : 0.0);
    for (int64_t t = 0; t < k; ++t) F[zci[j * k + t]] += w * (double)zval[j * k + t];
  }
}

// New row i: u = z_i + lr F in FP64, rounded to FP32; the k columns of
// largest |u| (ties: lower column), written sorted by column.
void oracle_embed_select(int64_t d, int64_t k, const double* zi, const double* F, double lr, int32_t* out_ci,
                         float* out_val) {
  std::vector<float> u(d);
  for (int64_t c = 0; c < d; ++c) u[c] = (float)(zi[c] + lr * F[c]);
  std::vector<int32_t> order(d);
  for (int64_t c = 0; c < d; ++c) order[c] = (int32_t)c;
  std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const float ax = std::fabs(u[x]), ay = std::fabs(u[y]);
    return ax != ay ? ax > ay : x < y;
  });
  std::vector<int32_t> keep(order.begin(), order.begin() + k);
  std::sort(keep.begin(), keep.end());
  for (int64_t t = 0; t < k; ++t) {
    out_ci[t] = keep[t];
    out_val[t] = u[keep[t]];
  }
}

// Rows [row_begin, row_end) updated in minibatches of `batch` rows, in row
// order; zci / zval (n x k) are updated in place. Returns 0, or 1 on bad
// arguments.
int oracle_embed_epoch(int64_t n, const int32_t* arp, const int32_t* aci, const float* aval, int64_t d, int64_t k,
                       int32_t* zci, float* zval, double lr, int64_t batch, int64_t row_begin, int64_t row_end) {
  if (k < 1 || k > d || batch < 1 || row_begin < 0 || row_end > n || row_begin > row_end) return 1;
  std::vector<double> F(d), zi(d);
  for (int64_t r0 = row_begin; r0 < row_end; r0 += batch) {
    const int64_t r1 = std::min(row_end, r0 + batch);
    std::vector<int32_t> new_ci((r1 - r0) * k);
    std::vector<float> new_val((r1 - r0) * k);
    for (int64_t i = r0; i < r1; ++i) {  // every row reads the embedding as of r0
      oracle_embed_force(arp, aci, aval, d, k, zci, zval, i, F.data());
      std::fill(zi.begin(), zi.end(), 0.0);
      for (int64_t t = 0; t < k; ++t) zi[zci[i * k + t]] = zval[i * k + t];
      oracle_embed_select(d, k, zi.data(), F.data(), lr, &new_ci[(i - r0) * k], &new_val[(i - r0) * k]);
    }
    std::copy(new_ci.begin(), new_ci.end(), zci + r0 * k);
    std::copy(new_val.begin(), new_val.end(), zval + r0 * k);
  }
  return 0;
}

// ---------------------------------------------------------------- tiles and merge

// Columns [c0, c1) of A, column ids kept: the tile of Sec. III-B taken over
// the full height. out_rp (n + 1) is filled; returns nnz, and fills out_ci /
// out_val when they are non-null.
int64_t oracle_column_slice(int64_t n, const int32_t* arp, const int32_t* aci, const double* aval, int32_t c0,
                            int32_t c1, int64_t* out_rp, int32_t* out_ci, double* out_val) {
  int64_t q = 0;
  out_rp[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int32_t p = arp[i]; p < arp[i + 1]; ++p)
      if (aci[p] >= c0 && aci[p] < c1) {
        if (out_ci) out_ci[q] = aci[p];
        if (out_val) out_val[q] = aval ? aval[p] : 0.0;
        ++q;
      }
    out_rp[i + 1] = q;
  }
  return q;
}

// Merge of partial outputs (Algorithm 2, Merge): the sum of `count` n-row
// CSR matrices, row by row, adding the parts in order in FP64.
void* oracle_merge_rows(int64_t n, int32_t count, const int32_t* const* rps, const int32_t* const* cis,
                        const double* const* vals) {
  Rows* r = new Rows;
  r->rp.assign(n + 1, 0);
  std::vector<std::map<int32_t, double>> acc(n);
  for (int32_t t = 0; t < count; ++t)
    for (int64_t i = 0; i < n; ++i)
      for (int32_t p = rps[t][i]; p < rps[t][i + 1]; ++p) acc[i][cis[t][p]] += vals[t][p];
  for (int64_t i = 0; i < n; ++i) {
    r->rp[i + 1] = r->rp[i] + (int64_t)acc[i].size();
    for (auto& kv : acc[i]) {
      r->ci.push_back(kv.first);
      r->val.push_back(kv.second);
    }
  }
  return r;
}

}  // extern "C"
