// Host-side state shared by the C-ABI translation units.
#pragma once

#include <mutex>

#include "core.hpp"

namespace tss {

// Grow-only device buffer; owns its allocation (move-only).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), cap(o.cap) {
    o.p = nullptr;
    o.cap = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      cap = o.cap;
      o.p = nullptr;
      o.cap = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  int ensure(size_t bytes);
  void release();
};

struct Plan {
  int dev = 0;
  int sr = 0;
  int64_t n = 0, d = 0;
  int wp = 1;
  int64_t a_nnz = 0, b_nnz = 0;
  tsspgemm_tuning tune{};
  bool ready = false;
  int32_t* crp = nullptr;  // caller's C row pointers (from the symbolic call)
  // device workspace
  DevBuf bbits, cbits, flops, cnt, scan, sym_items, num_items, split_rows, partial, ctr, maskbits;
  DevBuf gb_items, gb_split, gb_partial, gb_ctr;  // dL/dB work lists
  DevBuf bcol;             // B's column ids narrowed to col_id_bytes(d) bytes (numeric phase)
  DevBuf ebnd;             // per A entry, its B row's bounds (int2), recorded by the second numeric call
  bool ebnd_valid = false; //   of the plan (run_numeric); read by later calls and the backward
  int numeric_calls = 0;   // numeric calls since the plan's symbolic phase
  // dL/dB from sampled G: one block per A entry (i,k) holding A(i,k) and
  // G(i, pat(B_k)) in a 64-byte-multiple slot, blocks in A^T order; the start
  // of each B row's blocks and of each A entry's block, and the per-row sizes
  // and scan space that build them (built once per plan: the patterns are
  // fixed)
  DevBuf gb_gbuf, gb_off, gb_slot_a, gb_words, gb_scan;
  bool gb_pos_ready = false;
  bool gb_items_ready = false;  // the dL/dB work list (gb_items, gb_split, gb_ctr) is built
  int64_t gb_total = 0;     // products of the plan = entries of gb_gbuf (the last block start)
  bool masked = false;     // symbolic phase ran with a complement mask
  bool hash = false;       // hash accumulator plan (no bitmaps, no work lists)
  DevBuf hmask_rp, hmask_ci, hmask_bits;  // hash plan: copy of the complement mask
  HashMask hmask{};
  DevBuf hstrips;          // hash plan: private d-wide strips of the long-row kernel (kept zero)
  DevBuf hnext;            // hash plan: row counter of the long-row workers
  // hash plan, split rows: slot of each row, row of each slot, chunk list,
  // bitmaps, per-word counts, accumulator offsets, accumulators
  DevBuf hs_slot, hs_rows, hs_items, hs_bits, hs_pref, hs_off, hs_acc, hs_wins;
  DevBuf hs_cls, hs_cls_cnt;  // hash plan: row lists of the LDS table size classes, and their counts
  DevBuf hs_chunk_lists;      // hash plan: split-row chunks by class
  int64_t hs_item_cap = 0;
  int32_t hs_cls_host[6] = {0, 0, 0, 0, 0, 0};
  int64_t hs_cap = 0, hs_rows_n = 0, hs_items_n = 0, hs_acc_n = 0, hs_win_n = 0, hs_split_flops = 0;
  bool hs_all_split = false;  // every row with kHashSplitMin products or more is split
  DevBuf sp_chunks, sp_rows, sp_partial, sp_ctr;  // dense-B SpMM workspace (per-device cached plan)
  DevBuf em_ci, em_val;    // embedding update: second copy of Z (per-device cached plan)
  DevBuf em_cnt, em_split, em_slot_off, em_split_off, em_slot_row, em_split_list, em_partial, em_scan;
  DevBuf em_done;          // embedding update: finished chunks of each long row
  size_t hstrips_zeroed = 0;
  hipEvent_t ord_ev = nullptr;     // cached plans: end of the last call (see order_after_last)
  hipStream_t ord_last = nullptr;  //   and its stream
  bool ord_valid = false;
  Counters* host_ctr = nullptr;  // pinned
  // symbolic phase: a second stream of the plan (default priority) for the
  // work that does not wait for B's bitmap, and its fork / join events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_bm = nullptr, ev_join = nullptr;
  // results of the last symbolic call
  int64_t nnz = 0, flops_total = 0, n_split_items = 0, n_block_items = 0, n_wave_rows = 0, n_light_rows = 0;
  int64_t n_split_rows = 0;
  std::mutex mu;
  ~Plan() {
    if (host_ctr) (void)hipHostFree(host_ctr);
    host_ctr = nullptr;
    if (ord_ev) (void)hipEventDestroy(ord_ev);
    for (hipEvent_t e : {ev_fork, ev_bm, ev_join})
      if (e) (void)hipEventDestroy(e);
    if (side) (void)hipStreamDestroy(side);
  }
};

int check_csr(const tsspgemm_csr* m, const char* name, bool need_vals);
bool validate_enabled();
int validate_on_device(const tsspgemm_csr* m, const char* name, Counters* dctr, Counters* hctr, hipStream_t st);
void resolve_tuning(const tsspgemm_tuning* t, const tsspgemm_csr* B, tsspgemm_tuning* out);
int32_t sym_split_default(int wp, bool stops_early);
int run_symbolic(Plan* p, const tsspgemm_csr* A, const tsspgemm_csr* B, int sr, const tsspgemm_mask* M,
                 const tsspgemm_tuning* tune, int32_t* c_rowptr, int64_t* c_nnz, hipStream_t st);
int run_numeric(Plan* p, const tsspgemm_csr* A, const tsspgemm_csr* B, int32_t* c_colidx, void* c_vals,
                hipStream_t st);
void plan_free(Plan* p);
Plan* cached_plan(int dev);  // workspace of the one-shot entry points, per device
// Cross-stream ordering of the calls that share a cached plan: call
// order_after_last before queuing a call's work and mark_done after.
int order_after_last(Plan* p, hipStream_t st);
int mark_done(Plan* p, hipStream_t st);
// Scope of one call on a cached plan (held under the plan's mutex): waits
// for the previous call on another stream, records this call's end when the
// scope closes (also on an error return, for whatever was queued).
struct StreamOrder {
  Plan* p;
  hipStream_t st;
  int rc;
  StreamOrder(Plan* p_, hipStream_t st_) : p(p_), st(st_), rc(order_after_last(p_, st_)) {}
  ~StreamOrder() { (void)mark_done(p, st); }
  StreamOrder(const StreamOrder&) = delete;
  StreamOrder& operator=(const StreamOrder&) = delete;
};

}  // namespace tss
