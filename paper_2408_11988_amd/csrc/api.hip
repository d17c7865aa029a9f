// C ABI of the TS-SpGEMM library: argument checks, plans and their device
// workspace, and the ordering of the kernels of each call. Declarations and
// contracts are in include/tsspgemm.h.
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "api_internal.hpp"

namespace tss {

// True while `st` is capturing into a graph.
static bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const std::string& get_error() { return g_last_error; }

int DevBuf::ensure(size_t bytes) {
  if (bytes <= cap) return TSSPGEMM_OK;
  if (p) {
    hipError_t e = hipFree(p);
    p = nullptr;
    cap = 0;
    if (e != hipSuccess) {
      set_error(std::string("hipFree: ") + hipGetErrorString(e));
      return TSSPGEMM_ERR_HIP;
    }
  }
  size_t want = bytes < 256 ? 256 : bytes;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    set_error("device workspace allocation of " + std::to_string(want) + " bytes failed: " + hipGetErrorString(e));
    return TSSPGEMM_ERR_NOMEM;
  }
  cap = want;
  return TSSPGEMM_OK;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
}

bool validate_enabled() {
  const char* v = std::getenv("TSSPGEMM_VALIDATE");
  return v && v[0] == '1';
}

int check_csr(const tsspgemm_csr* m, const char* name, bool need_vals) {
  if (!m) {
    set_error(std::string(name) + " is NULL");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (m->nrows < 0 || m->ncols < 0 || m->nnz < 0) {
    set_error(std::string(name) + ": negative shape or nnz");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (m->nrows > INT32_MAX - 1 || m->ncols > INT32_MAX || m->nnz > INT32_MAX) {
    set_error(std::string(name) + ": shape or nnz exceeds int32 indexing");
    return TSSPGEMM_ERR_OVERFLOW;
  }
  if (!m->rowptr || (m->nnz > 0 && !m->colidx) || (need_vals && m->nnz > 0 && !m->vals)) {
    set_error(std::string(name) + ": NULL array");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  return TSSPGEMM_OK;
}

// Device check of CSR invariants (only with TSSPGEMM_VALIDATE=1); synchronizes.
int validate_on_device(const tsspgemm_csr* m, const char* name, Counters* dctr, Counters* hctr, hipStream_t st) {
  int rc = launch_zero_bytes(dctr, sizeof(Counters), st);
  if (rc) return rc;
  rc = launch_validate_csr(m->nrows, m->ncols, m->nnz, m->rowptr, m->colidx, dctr, st);
  if (rc) return rc;
  TSS_HIP(hipMemcpyAsync(hctr, dctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  TSS_HIP(hipStreamSynchronize(st));
  if (hctr->malformed) {
    set_error(std::string(name) + ": malformed CSR (row pointers or sorted unique in-range columns)");
    return TSSPGEMM_ERR_MALFORMED;
  }
  return TSSPGEMM_OK;
}

static int plan_alloc_host(Plan* p) {
  if (p->host_ctr) return TSSPGEMM_OK;
  void* h = nullptr;
  TSS_HIP(hipHostMalloc(&h, sizeof(Counters), hipHostMallocDefault));
  p->host_ctr = (Counters*)h;
  return TSSPGEMM_OK;
}

void plan_free(Plan* p) {
  for (DevBuf* b : {&p->bbits, &p->cbits, &p->flops, &p->cnt, &p->scan, &p->sym_items, &p->num_items,
                    &p->split_rows, &p->partial, &p->ctr, &p->maskbits, &p->gb_items, &p->gb_split,
                    &p->gb_partial, &p->gb_ctr, &p->gb_gbuf, &p->gb_off, &p->gb_slot_a, &p->gb_words, &p->gb_scan,
                    &p->ebnd})
    b->release();
  if (p->host_ctr) (void)hipHostFree(p->host_ctr);
  p->host_ctr = nullptr;
  p->hstrips_zeroed = 0;
}

// Lanes per B row: the smallest power of two (8..64) covering the mean B row
// length, so a B row is mostly read in one step. Measured on R-MAT at 1.9,
// 2.6, 12.8, 25.6 and 64 entries per B row (8, 8, 16, 32 and 64 lanes best
// with per-B-row products).
int default_group_lanes(double mean_b_row) {
  int gl = 8;
  while (gl < 64 && gl < mean_b_row) gl <<= 1;
  return gl;
}

static double mean_b_row(const tsspgemm_csr* B) { return B->nrows > 0 ? (double)B->nnz / (double)B->nrows : 0.0; }

// Flat product lists for long B rows (a lane then has several independent
// loads per step where a per-B-row group would walk the row's tail serially);
// per B row otherwise, since a lane of the flat layout walks the staged
// entries and short rows make that walk long.
int default_products(double mean_b_row, int group_lanes) {
  (void)group_lanes;
  return mean_b_row >= 48.0 ? TSSPGEMM_PRODUCTS_FLAT : TSSPGEMM_PRODUCTS_PER_B_ROW;
}

// Entries per symbolic chunk of a split row when the caller leaves it open.
// Heavy kernels that stop once a row's pattern is full (the unmasked lane
// form, bitmaps of at most 8 words) take 8192: at R-MAT 20 x 128 the pass
// takes 0.345 / 0.343 / 0.336 / 0.362 ms with 2048 / 4096 / 8192 / 16384
// (with the heavy walk on eight times the resident wavefronts, 4096 and
// 8192 tie at 0.314 and 16384 takes 0.320). The BFS, whose items stop once
// their open columns are covered, takes 16384: R-MAT 22 x 512 in 14.6-14.7
// ms, against 14.9 with 8192 and 4096. The others walk every entry, some 8
// per step (the slot form at d > 512), and keep 2048: 8192 took the R-MAT
// 18 x 1024 pass from 0.51 to 1.03 ms.
int32_t sym_split_default(int wp, bool stops_early) { return stops_early ? 16384 : (wp <= 8 ? 8192 : 2048); }

void resolve_tuning(const tsspgemm_tuning* t, const tsspgemm_csr* B, tsspgemm_tuning* out) {
  tsspgemm_tuning r{};
  if (t) r = *t;
  // lanes per B row: 4-entry chunks per lane need a quarter of the lanes
  if (r.group_lanes == 0)
    r.group_lanes = default_group_lanes(r.products == TSSPGEMM_PRODUCTS_VEC4 ? mean_b_row(B) / 4.0 : mean_b_row(B));
  if (r.light_max_flops <= 0) r.light_max_flops = 1024;
  if (r.wave_max_flops <= 0) r.wave_max_flops = 65536;
  if (r.split_flops <= 0) r.split_flops = 262144;
  if (r.wave_max_flops < r.light_max_flops) r.wave_max_flops = r.light_max_flops;
  if (r.split_flops < r.wave_max_flops) r.split_flops = r.wave_max_flops;
  // symbolic chunks of split rows (larger ones where the heavy kernel stops
  // early: see sym_split_default)
  if (r.sym_split_nnz <= 0) r.sym_split_nnz = 2048;
  if (r.products == TSSPGEMM_PRODUCTS_AUTO) r.products = default_products(mean_b_row(B), r.group_lanes);
  if (r.accumulator == TSSPGEMM_ACC_AUTO)
    r.accumulator = B->ncols > kMaxDenseD ? TSSPGEMM_ACC_HASH : TSSPGEMM_ACC_LDS_STRIP;
  *out = r;
}

// Symbolic phase with the hash accumulator: per-row distinct-column counts
// (k_hash.hip), then the same count scan as the bitmap path. The mask is
// copied into the plan, since the numeric phase tests it again.
static HashSplit hash_split_view(Plan* p) {
  HashSplit hs{};
  hs.slot_of_row = (int32_t*)p->hs_slot.p;
  hs.rows = (int32_t*)p->hs_rows.p;
  hs.items = (int2*)p->hs_items.p;
  hs.bits = (uint32_t*)p->hs_bits.p;
  hs.pref = (int32_t*)p->hs_pref.p;
  hs.acc_off = (int32_t*)p->hs_off.p;
  hs.acc = p->hs_acc.p;
  hs.wins = (int2*)p->hs_wins.p;
  hs.cls_rows = (int32_t*)p->hs_cls.p;
  hs.cls_cnt = (int32_t*)p->hs_cls_cnt.p;
  hs.chunk_lists = (int32_t*)p->hs_chunk_lists.p;
  hs.item_cap = (int32_t)p->hs_item_cap;
  hs.cap = (int32_t)p->hs_cap;
  hs.split_flops = p->hs_split_flops;
  hs.ctr = (Counters*)p->ctr.p;
  return hs;
}

static int run_symbolic_hash(Plan* p, const tsspgemm_csr* A, const tsspgemm_csr* B, int sr, const tsspgemm_mask* M,
                             const tsspgemm_tuning& tn, int32_t* c_rowptr, int64_t* c_nnz, hipStream_t st) {
  int rc;
  const int64_t n = A->nrows, d = B->ncols;
  p->n = n;
  p->d = d;
  p->wp = bitmap_words((int32_t)(d < 1 ? 1 : d));
  p->sr = sr;
  p->tune = tn;
  p->tune.accumulator = TSSPGEMM_ACC_HASH;
  p->crp = c_rowptr;
  p->a_nnz = A->nnz;
  p->b_nnz = B->nnz;
  p->ready = false;
  p->gb_pos_ready = false;
  p->gb_items_ready = false;
  p->hash = true;
  p->ebnd_valid = false;
  p->masked = M && M->kind != TSSPGEMM_MASK_NONE;
  if ((rc = plan_alloc_host(p))) return rc;
  if ((rc = p->ctr.ensure(sizeof(Counters))) || (rc = p->flops.ensure((size_t)n * 8)) ||
      (rc = p->cnt.ensure((size_t)n * 4)) || (rc = p->scan.ensure((size_t)scan_block_sums_capacity(n) * 8)))
    return rc;
  Counters* ctr = (Counters*)p->ctr.p;
  if (validate_enabled()) {
    if ((rc = validate_on_device(A, "A", ctr, p->host_ctr, st)) || (rc = validate_on_device(B, "B", ctr, p->host_ctr, st)))
      return rc;
    if (M && M->kind == TSSPGEMM_MASK_COMPLEMENT_CSR && (rc = validate_on_device(M->csr, "mask", ctr, p->host_ctr, st)))
      return rc;
  }
  p->hmask = HashMask{};
  if (M && M->kind == TSSPGEMM_MASK_COMPLEMENT_CSR) {
    const tsspgemm_csr* m = M->csr;
    if ((rc = p->hmask_rp.ensure((size_t)(n + 1) * 4)) || (rc = p->hmask_ci.ensure((size_t)m->nnz * 4))) return rc;
    TSS_HIP(hipMemcpyAsync(p->hmask_rp.p, m->rowptr, (size_t)(n + 1) * 4, hipMemcpyDeviceToDevice, st));
    if (m->nnz > 0)
      TSS_HIP(hipMemcpyAsync(p->hmask_ci.p, m->colidx, (size_t)m->nnz * 4, hipMemcpyDeviceToDevice, st));
    p->hmask.rp = (const int32_t*)p->hmask_rp.p;
    p->hmask.ci = (const int32_t*)p->hmask_ci.p;
  } else if (M && M->kind == TSSPGEMM_MASK_COMPLEMENT_BITMAP) {
    const size_t bytes = (size_t)n * p->wp * 4;
    if ((rc = p->hmask_bits.ensure(bytes))) return rc;
    if (bytes) TSS_HIP(hipMemcpyAsync(p->hmask_bits.p, M->bits, bytes, hipMemcpyDeviceToDevice, st));
    p->hmask.bits = (const uint32_t*)p->hmask_bits.p;
    p->hmask.wpm = p->wp;
  }
  Problem pr{};
  pr.n = (int32_t)n;
  pr.d = (int32_t)d;
  pr.wp = p->wp;
  pr.arp = A->rowptr;
  pr.aci = A->colidx;
  pr.brp = B->rowptr;
  pr.bci = B->colidx;
  pr.flops = (int64_t*)p->flops.p;
  pr.crp = c_rowptr;
  if ((rc = launch_zero_bytes(ctr, sizeof(Counters), st))) return rc;
  // products per row and their histogram first: the split threshold and the
  // split slots follow from it
  if ((rc = launch_hash_flops(pr, ctr->hash_hist, st))) return rc;
  TSS_HIP(hipMemcpyAsync(p->host_ctr, ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  TSS_HIP(hipStreamSynchronize(st));
  const int64_t words = (d + 31) / 32;
  hash_split_choose(p->host_ctr->hash_hist, d < 1 ? 1 : d, &p->hs_split_flops, &p->hs_cap);
  const int64_t item_cap = hash_split_item_cap(A->nnz, p->hs_cap);
  p->hs_item_cap = item_cap;
  if ((rc = p->hs_slot.ensure((size_t)n * 4)) || (rc = p->hs_rows.ensure((size_t)p->hs_cap * 4)) ||
      (rc = p->hs_items.ensure((size_t)item_cap * 8)) || (rc = p->hs_bits.ensure((size_t)p->hs_cap * words * 4)) ||
      (rc = p->hs_pref.ensure((size_t)p->hs_cap * words * 4)) || (rc = p->hs_off.ensure((size_t)p->hs_cap * 4)) ||
      (rc = p->hs_wins.ensure((size_t)hash_split_window_cap(p->hs_cap, d < 1 ? 1 : d) * 8)) ||
      (rc = p->hs_cls.ensure((size_t)n * 16)) || (rc = p->hs_cls_cnt.ensure(24)) ||
      (rc = p->hs_chunk_lists.ensure((size_t)item_cap * 8)))
    return rc;
  const HashSplit hs = hash_split_view(p);
  // every candidate split: the rows left have fewer than kHashSplitMin products
  p->hs_all_split = p->hs_cap == hash_split_candidates(p->host_ctr->hash_hist);
  if ((rc = launch_hash_symbolic(pr, p->hmask, hs, p->hs_all_split, (int32_t*)p->cnt.p, &ctr->hash_error, st)))
    return rc;
  pr.cbits = nullptr;  // counts come from cnt
  if ((rc = launch_count_scan(pr, (int32_t*)p->cnt.p, (int64_t*)p->scan.p, c_rowptr, ctr, st))) return rc;
  TSS_HIP(hipMemcpyAsync(p->host_ctr, ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  if (n > 0) TSS_HIP(hipMemcpyAsync(p->hs_cls_host, p->hs_cls_cnt.p, 24, hipMemcpyDeviceToHost, st));
  TSS_HIP(hipStreamSynchronize(st));
  if (n == 0)
    for (int c = 0; c < 6; ++c) p->hs_cls_host[c] = 0;
  const Counters& h = *p->host_ctr;
  if (h.hash_error) {
    set_error("hash accumulator: inconsistent row table");
    return TSSPGEMM_ERR_HIP;
  }
  p->nnz = h.nnz_total;
  p->flops_total = h.flops_total;
  p->n_split_items = p->n_block_items = p->n_wave_rows = p->n_light_rows = p->n_split_rows = 0;
  p->hs_rows_n = h.hash_split_rows < p->hs_cap ? h.hash_split_rows : p->hs_cap;
  p->hs_items_n = h.hash_split_items;
  p->hs_acc_n = h.hash_split_acc;
  p->hs_win_n = h.hash_win_items;
  p->n_split_rows = p->hs_rows_n;
  p->n_split_items = p->hs_items_n;
  *c_nnz = h.nnz_total;
  if (h.nnz_total > INT32_MAX) {
    set_error("nnz(C) = " + std::to_string(h.nnz_total) + " exceeds INT32_MAX");
    return TSSPGEMM_ERR_OVERFLOW;
  }
  if (sr != TSSPGEMM_OR_AND && p->hs_acc_n > 0 &&
      (rc = p->hs_acc.ensure((size_t)p->hs_acc_n * (sr == TSSPGEMM_PLUS_TIMES_F32 ? 8 : 4))))
    return rc;
  if (sr != TSSPGEMM_OR_AND && n > 0) {
    const size_t bytes = (size_t)hash_dense_workers(d) * d * (sr == TSSPGEMM_PLUS_TIMES_F32 ? 8 : 4);
    if ((rc = p->hstrips.ensure(bytes))) return rc;
    if (p->hstrips_zeroed < bytes) {  // the long-row kernel leaves its strips all-zero
      if ((rc = launch_zero_bytes(p->hstrips.p, bytes, st))) return rc;
      p->hstrips_zeroed = bytes;
    }
  }
  p->ready = true;
  return TSSPGEMM_OK;
}

// Symbolic phase shared by tsspgemm_symbolic and tsspgemm_masked_bool.
int run_symbolic(Plan* p, const tsspgemm_csr* A, const tsspgemm_csr* B, int sr, const tsspgemm_mask* M,
                 const tsspgemm_tuning* tune, int32_t* c_rowptr, int64_t* c_nnz, hipStream_t st) {
  int rc;
  if ((rc = check_csr(A, "A", false)) || (rc = check_csr(B, "B", false))) return rc;
  if (A->nrows != A->ncols) {
    set_error("A must be square (n x n)");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (B->nrows != A->ncols) {
    set_error("B must have as many rows as A has columns");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (!c_rowptr || !c_nnz) {
    set_error("c_rowptr and c_nnz must not be NULL");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (sr < 0 || sr > 2) {
    set_error("unknown semiring");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (M && M->kind != TSSPGEMM_MASK_NONE) {
    if (M->kind == TSSPGEMM_MASK_COMPLEMENT_CSR) {
      if ((rc = check_csr(M->csr, "mask", false))) return rc;
      if (M->csr->nrows != A->nrows || M->csr->ncols != B->ncols) {
        set_error("mask must be n x d");
        return TSSPGEMM_ERR_INVALID_ARG;
      }
    } else if (M->kind == TSSPGEMM_MASK_COMPLEMENT_BITMAP) {
      if (!M->bits && A->nrows > 0) {
        set_error("bitmap mask without bits");
        return TSSPGEMM_ERR_INVALID_ARG;
      }
    } else {
      set_error("unknown mask kind");
      return TSSPGEMM_ERR_INVALID_ARG;
    }
  }
  tsspgemm_tuning tn;
  resolve_tuning(tune, B, &tn);
  if (!(tune && tune->sym_split_nnz > 0))  // masked passes take the lane form with the mask, which walks every entry
    tn.sym_split_nnz = sym_split_default(M && M->kind != TSSPGEMM_MASK_NONE ? 16 : bitmap_words((int32_t)B->ncols), false);
  if (tn.accumulator != TSSPGEMM_ACC_LDS_STRIP && tn.accumulator != TSSPGEMM_ACC_HASH) {
    set_error("unknown accumulator");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (tn.products != TSSPGEMM_PRODUCTS_PER_B_ROW && tn.products != TSSPGEMM_PRODUCTS_FLAT &&
      tn.products != TSSPGEMM_PRODUCTS_VEC4) {
    set_error("unknown product layout");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (B->ncols > kMaxDenseD && tn.accumulator == TSSPGEMM_ACC_LDS_STRIP) {
    set_error("the LDS strip accumulator needs d <= 1024");
    return TSSPGEMM_ERR_UNSUPPORTED;
  }
  if (B->ncols > kMaxDenseD || tn.accumulator == TSSPGEMM_ACC_HASH) {
    if (B->ncols > kHashMaxD) {
      set_error("d > " + std::to_string(kHashMaxD) + " is not supported");
      return TSSPGEMM_ERR_UNSUPPORTED;
    }
    return run_symbolic_hash(p, A, B, sr, M, tn, c_rowptr, c_nnz, st);
  }
  p->hash = false;
  const int64_t n = A->nrows, d = B->ncols;
  const int wp = bitmap_words(d);
  p->n = n;
  p->d = d;
  p->wp = wp;
  p->sr = sr;
  p->tune = tn;
  p->crp = c_rowptr;
  p->a_nnz = A->nnz;
  p->b_nnz = B->nnz;
  p->ready = false;
  p->gb_pos_ready = false;
  p->gb_items_ready = false;
  p->masked = M && M->kind != TSSPGEMM_MASK_NONE;
  if ((rc = plan_alloc_host(p))) return rc;
  const int64_t sym_cap = n + A->nnz / tn.sym_split_nnz + 2;
  const int64_t num_cap = 2 * n + A->nnz / 64 + 2;
  if ((rc = p->ctr.ensure(sizeof(Counters))) || (rc = p->bbits.ensure((size_t)n * wp * 4)) ||
      (rc = p->cbits.ensure((size_t)n * wp * 4)) || (rc = p->flops.ensure((size_t)n * 8)) ||
      (rc = p->cnt.ensure((size_t)n * 4)) || (rc = p->scan.ensure((size_t)scan_block_sums_capacity(n) * 8)) ||
      (rc = p->sym_items.ensure((size_t)sym_cap * sizeof(Item))) ||
      (rc = p->num_items.ensure((size_t)num_cap * sizeof(Item))) ||
      (rc = p->split_rows.ensure((size_t)(n + 1) * sizeof(SplitRow))))
    return rc;
  Counters* ctr = (Counters*)p->ctr.p;

  if (validate_enabled()) {
    if ((rc = validate_on_device(A, "A", ctr, p->host_ctr, st)) || (rc = validate_on_device(B, "B", ctr, p->host_ctr, st)))
      return rc;
    if (M && M->kind == TSSPGEMM_MASK_COMPLEMENT_CSR && (rc = validate_on_device(M->csr, "mask", ctr, p->host_ctr, st)))
      return rc;
  }

  Problem pr{};
  pr.n = (int32_t)n;
  pr.d = (int32_t)d;
  pr.wp = wp;
  pr.arp = A->rowptr;
  pr.aci = A->colidx;
  pr.aval = A->vals;
  pr.brp = B->rowptr;
  pr.bci = B->colidx;
  pr.bval = B->vals;
  pr.bbits = (const uint32_t*)p->bbits.p;
  pr.cbits = (uint32_t*)p->cbits.p;
  pr.flops = (int64_t*)p->flops.p;
  pr.crp = c_rowptr;
  p->ebnd_valid = false;  // new patterns: the B row bounds are recorded again (run_numeric)
  p->numeric_calls = 0;

  if ((rc = launch_zero_bytes(ctr, sizeof(Counters), st))) return rc;
  // Two streams: the binning of A's rows (it does not need B; split rows'
  // bitmap rows and counts are cleared there too) and then the heavy items
  // run on the plan's side stream, while `stream` builds B's bitmap and then
  // walks the light rows; the heavy items wait for the bitmap, and `stream`
  // waits for the heavy items before the counts. (Each wait across the
  // streams costs about 10 us on the device, so there is one each way.)
  if (!p->side) TSS_HIP(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
  for (hipEvent_t* e : {&p->ev_fork, &p->ev_bm, &p->ev_join})
    if (!*e) TSS_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  TSS_HIP(hipEventRecord(p->ev_fork, st));
  TSS_HIP(hipStreamWaitEvent(p->side, p->ev_fork, 0));
  if ((rc = launch_sym_bin(pr, tn.sym_split_nnz, (Item*)p->sym_items.p, ctr, p->side, true))) return rc;
  // B's bitmap; for value semirings the same pass narrows B's column ids
  // (the numeric phase reads them; B's pattern is fixed for the plan)
  const int cb = sr != TSSPGEMM_OR_AND ? col_id_bytes(d) : 0;
  if (cb && (rc = p->bcol.ensure((size_t)B->nnz * cb))) return rc;
  if ((rc = launch_csr_to_bitmap(n, B->rowptr, B->colidx, wp, (uint32_t*)p->bbits.p, st, cb ? p->bcol.p : nullptr,
                                 cb)))
    return rc;
  const uint32_t* mask = nullptr;
  if (M && M->kind == TSSPGEMM_MASK_COMPLEMENT_CSR) {
    if ((rc = p->maskbits.ensure((size_t)n * wp * 4))) return rc;
    if ((rc = launch_csr_to_bitmap(n, M->csr->rowptr, M->csr->colidx, wp, (uint32_t*)p->maskbits.p, st))) return rc;
    mask = (const uint32_t*)p->maskbits.p;
  } else if (M && M->kind == TSSPGEMM_MASK_COMPLEMENT_BITMAP) {
    mask = M->bits;
  }
  SymParams sp{};
  sp.pr = pr;
  sp.items = (const Item*)p->sym_items.p;
  sp.ctr = ctr;
  sp.mask = mask;
  TSS_HIP(hipEventRecord(p->ev_bm, st));
  if ((rc = launch_symbolic_part(sp, sym_cap, kSymLight, st))) return rc;
  TSS_HIP(hipStreamWaitEvent(p->side, p->ev_bm, 0));
  if ((rc = launch_symbolic_part(sp, sym_cap, kSymHeavy, p->side))) return rc;
  TSS_HIP(hipEventRecord(p->ev_join, p->side));
  TSS_HIP(hipStreamWaitEvent(st, p->ev_join, 0));
  if ((rc = launch_sym_split_mask(pr, (const Item*)p->sym_items.p, mask, ctr, sym_cap, st))) return rc;
  // the numeric phase's work binning (value semirings) rides on the count
  // and row-pointer passes over the rows
  const NumBinArgs nb{NumThresholds{tn.light_max_flops, tn.wave_max_flops, tn.split_flops}, (Item*)p->num_items.p,
                      (SplitRow*)p->split_rows.p};
  if ((rc = launch_count_scan(pr, (int32_t*)p->cnt.p, (int64_t*)p->scan.p, c_rowptr, ctr, st,
                              sr != TSSPGEMM_OR_AND ? &nb : nullptr)))
    return rc;
  TSS_HIP(hipMemcpyAsync(p->host_ctr, ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  TSS_HIP(hipStreamSynchronize(st));
  const Counters& h = *p->host_ctr;
  p->nnz = h.nnz_total;
  p->flops_total = h.flops_total;
  p->n_split_items = h.num_split_items;
  p->n_block_items = h.num_block_items;
  p->n_wave_rows = h.num_wave_rows;
  p->n_light_rows = h.num_light_rows;
  p->n_split_rows = h.num_split_rows;
  *c_nnz = h.nnz_total;
  if (h.nnz_total > INT32_MAX) {
    set_error("nnz(C) = " + std::to_string(h.nnz_total) + " exceeds INT32_MAX");
    return TSSPGEMM_ERR_OVERFLOW;
  }
  if (sr != TSSPGEMM_OR_AND && p->n_split_items > 0) {
    const size_t esz = sr == TSSPGEMM_PLUS_TIMES_F32 ? 8 : 4;
    if ((rc = p->partial.ensure((size_t)p->n_split_items * d * esz))) return rc;
  }
  p->ready = true;
  return TSSPGEMM_OK;
}

int run_numeric(Plan* p, const tsspgemm_csr* A, const tsspgemm_csr* B, int32_t* c_colidx, void* c_vals,
                hipStream_t st) {
  int rc;
  if (!p || !p->ready) {
    set_error("numeric: plan is NULL or its symbolic phase did not succeed");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  const bool vals = p->sr != TSSPGEMM_OR_AND;
  if ((rc = check_csr(A, "A", vals)) || (rc = check_csr(B, "B", vals))) return rc;
  if (A->nrows != p->n || B->ncols != p->d || A->nnz != p->a_nnz || B->nnz != p->b_nnz) {
    set_error("numeric: A or B differs in shape or nnz from the plan's symbolic call");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (p->nnz > 0 && (!c_colidx || (vals && !c_vals))) {
    set_error("numeric: NULL output array");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
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
  pr.cci = c_colidx;
  pr.cval = c_vals;
  if (p->nnz == 0) return TSSPGEMM_OK;
  if (p->hash) {
    if ((rc = p->hnext.ensure(64))) return rc;
    return launch_hash_numeric(p->sr, pr, p->hmask, hash_split_view(p), (int32_t)p->hs_rows_n,
                               (int32_t)p->hs_items_n, p->hs_acc_n, (int32_t)p->hs_win_n, p->hs_cls_host,
                               !p->hs_all_split, p->hstrips.p,
                               &((Counters*)p->ctr.p)->hash_error, (int32_t*)p->hnext.p, st);
  }
  if (!vals) return launch_emit_pattern(pr, st);
  // A plan whose numeric phase repeats (a training loop): the second call
  // records each A entry's B row bounds as its staging gathers them (8 B per
  // A entry), and later calls and the backward read them instead. A call
  // being captured into a graph neither records nor counts: its kernels run
  // only when the graph is replayed, and the record's buffer may not be
  // allocated under capture.
  bool recording = false;
  if (p->ebnd_valid) {
    pr.ebnd = (const int2*)p->ebnd.p;
  } else if (!capturing(st) && ++p->numeric_calls >= 2) {
    if ((rc = p->ebnd.ensure((size_t)p->a_nnz * sizeof(int2)))) return rc;
    pr.ebnd_w = (int2*)p->ebnd.p;
    recording = true;
  }
  NumParams np{};
  np.pr = pr;
  np.items = (const Item*)p->num_items.p;
  np.n_wg_items = (int32_t)(p->n_split_items + p->n_block_items);
  np.n_heavy_records = (int32_t)(p->n_split_items + p->n_block_items + p->n_wave_rows);
  np.n_light = (int32_t)p->n_light_rows;
  np.pr.bcol = p->bcol.p;
  np.partial = (double*)p->partial.p;
  np.ipartial = (int32_t*)p->partial.p;
  const int64_t grid = np.n_wg_items + (p->n_wave_rows + kWavesPerBlock - 1) / kWavesPerBlock;
  // 4-entry chunks need B's values 16-byte aligned (the narrowed ids are the
  // plan's own, aligned); otherwise one entry per lane
  int products = p->tune.products;
  if (products == TSSPGEMM_PRODUCTS_VEC4 && ((uintptr_t)B->vals % 16) != 0) products = TSSPGEMM_PRODUCTS_PER_B_ROW;
  if ((rc = launch_numeric(p->sr, p->tune.group_lanes, products, np, grid, st))) return rc;
  if (recording) p->ebnd_valid = true;  // the staging of this call writes every staged entry's bounds
  return launch_split_finalize(p->sr, pr, (const SplitRow*)p->split_rows.p, (int32_t)p->n_split_rows,
                               (const double*)p->partial.p, (const int32_t*)p->partial.p, st);
}

// Workspaces of the one-shot entry points (masked_bool, spmm, embed_epoch),
// one per device, reused by every call on that device (also across a graph
// capture: the capture reuses what an eager call sized).
static std::mutex g_cache_mu;
static Plan* g_cache[64];

Plan* cached_plan(int dev) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (dev < 0 || dev >= 64) return nullptr;
  if (!g_cache[dev]) g_cache[dev] = new (std::nothrow) Plan();
  return g_cache[dev];
}

// Calls on different streams that share a cached workspace are ordered on
// the device: a call waits for the previous call's event when that call ran
// on another stream, and records its own at the end. Work being captured
// into a graph neither waits nor records (the caller orders graph replays).

int order_after_last(Plan* p, hipStream_t st) {
  if (!p->ord_valid || p->ord_last == st || capturing(st)) return TSSPGEMM_OK;
  TSS_HIP(hipStreamWaitEvent(st, p->ord_ev, 0));
  return TSSPGEMM_OK;
}

int mark_done(Plan* p, hipStream_t st) {
  if (capturing(st)) return TSSPGEMM_OK;
  if (!p->ord_ev) TSS_HIP(hipEventCreateWithFlags(&p->ord_ev, hipEventDisableTiming));
  TSS_HIP(hipEventRecord(p->ord_ev, st));
  p->ord_last = st;
  p->ord_valid = true;
  return TSSPGEMM_OK;
}

}  // namespace tss

using namespace tss;

extern "C" {

int32_t tsspgemm_bitmap_words(int32_t d) { return d < 0 ? 0 : bitmap_words(d); }

int tsspgemm_symbolic(const tsspgemm_csr* A, const tsspgemm_csr* B, int32_t sr, const tsspgemm_mask* M,
                      const tsspgemm_tuning* tune, int32_t* c_rowptr, int64_t* c_nnz, tsspgemm_plan* plan,
                      void* stream) {
  try {
    if (!plan) {
      set_error("plan must not be NULL");
      return TSSPGEMM_ERR_INVALID_ARG;
    }
    Plan* p = (Plan*)*plan;
    bool fresh = false;
    if (!p) {
      p = new (std::nothrow) Plan();
      if (!p) {
        set_error("out of host memory");
        return TSSPGEMM_ERR_NOMEM;
      }
      fresh = true;
    }
    (void)hipGetDevice(&p->dev);
    p->ready = false;
    int rc = run_symbolic(p, A, B, sr, M, tune, c_rowptr, c_nnz, (hipStream_t)stream);
    if (rc != TSSPGEMM_OK && fresh && rc != TSSPGEMM_ERR_OVERFLOW) {
      plan_free(p);
      delete p;
      return rc;
    }
    *plan = (tsspgemm_plan)p;
    return rc;
  } catch (...) {
    set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}

int tsspgemm_numeric(tsspgemm_plan plan, const tsspgemm_csr* A, const tsspgemm_csr* B, int32_t* c_colidx,
                     void* c_vals, void* stream) {
  try {
    return run_numeric((Plan*)plan, A, B, c_colidx, c_vals, (hipStream_t)stream);
  } catch (...) {
    set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}

int tsspgemm_plan_stats(tsspgemm_plan plan, int64_t* flops, int64_t* c_nnz, int64_t* light_rows, int64_t* wave_rows,
                        int64_t* block_rows, int64_t* split_rows) {
  Plan* p = (Plan*)plan;
  if (!p) {
    set_error("plan is NULL");
    return TSSPGEMM_ERR_INVALID_ARG;
  }
  if (flops) *flops = p->flops_total;
  if (c_nnz) *c_nnz = p->nnz;
  if (light_rows) *light_rows = p->n_light_rows;
  if (wave_rows) *wave_rows = p->n_wave_rows;
  if (block_rows) *block_rows = p->n_block_items;
  if (split_rows) *split_rows = p->n_split_rows;
  return TSSPGEMM_OK;
}

void tsspgemm_plan_destroy(tsspgemm_plan plan) {
  Plan* p = (Plan*)plan;
  if (!p) return;
  plan_free(p);
  delete p;
}

int tsspgemm_masked_bool(const tsspgemm_csr* A, const tsspgemm_csr* F, const tsspgemm_mask* visited,
                         int32_t* c_rowptr, int32_t* c_colidx, int64_t c_capacity, int64_t* c_nnz, void* stream) {
  try {
    int dev = 0;
    (void)hipGetDevice(&dev);
    Plan* p = cached_plan(dev);
    if (!p) {
      set_error("no plan cache for this device");
      return TSSPGEMM_ERR_NOMEM;
    }
    std::lock_guard<std::mutex> lk(p->mu);
    StreamOrder so(p, (hipStream_t)stream);
    if (so.rc) return so.rc;
    p->ready = false;
    int rc = run_symbolic(p, A, F, TSSPGEMM_OR_AND, visited, nullptr, c_rowptr, c_nnz, (hipStream_t)stream);
    if (rc) return rc;
    if (*c_nnz > c_capacity) {
      set_error("output capacity " + std::to_string(c_capacity) + " < nnz(C) = " + std::to_string(*c_nnz));
      return TSSPGEMM_ERR_CAPACITY;
    }
    return run_numeric(p, A, F, c_colidx, nullptr, (hipStream_t)stream);
  } catch (...) {
    set_error("unexpected C++ exception");
    return TSSPGEMM_ERR_HIP;
  }
}

const char* tsspgemm_last_error(void) { return get_error().c_str(); }

const char* tsspgemm_version(void) { return "tsspgemm-gfx950 0.1"; }

}  // extern "C"
