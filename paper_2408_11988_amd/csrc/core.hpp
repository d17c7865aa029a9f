// Internal interfaces between the C-ABI layer and the kernels.
#pragma once

#include "common.hpp"

namespace tss {

// A unit of row work: entries [p0, p1) of A's row `row`.
// aux: for symbolic items, kSplitFlag marks a chunk of a split row; for
// numeric split chunks, the index of the chunk's partial-sum slot.
struct Item {
  int32_t row, p0, p1, aux;
};
constexpr int32_t kSplitFlag = 1 << 30;
constexpr int32_t kNoSlot = 0x7fffffff;  // numeric workgroup item that is a whole row

constexpr int kBins = 32;  // work classes by floor(log2(work)); heavier first
// Binning kernels: a workgroup of 256 threads takes this many consecutive
// rows and makes one global reservation per bin for all of them (few
// workgroups, so few atomics on each bin counter).
constexpr int kBinRowsPerBlock = 4096;
constexpr int kNumClasses = 4;  // numeric: 0 split chunks, 1 workgroup rows, 2 wavefront rows, 3 light rows

// Rows with at most kSlotRowMax A entries ("light" rows, the bulk of a
// power-law graph) are processed straight from the row index, one row per
// lane or per slot of wp lanes. Heavier rows are binned into an item list
// (heaviest first) and take a whole wavefront, or several when split. The
// multi-source BFS takes rows of up to kSlotRowMaxBfs entries as light: its
// light rows stop early and skip the neighbours outside the frontier, so a
// lane can walk longer rows (R-MAT 22 x 512: 18.2 against 18.7 ms; the
// plain pass is fastest at 32: 0.345 ms, against 0.364 at 64 and 0.359 at 16).
constexpr int kSlotRowMax = 32;
constexpr int kSlotRowMaxBfs = 64;

// Product-count thresholds of the numeric work classes.
struct NumThresholds {
  int64_t light_max, wave_max, split;
};

// Device-side counters of one plan (zeroed by a kernel before each use).
struct Counters {
  int32_t sym_count[kBins];
  int32_t sym_cursor[kBins];
  int32_t num_count[kNumClasses][kBins];
  int32_t num_cursor[kNumClasses][kBins];
  int32_t sym_total;
  int32_t sym_split_rows;
  int32_t num_split_items;
  int32_t num_block_items;
  int32_t num_wave_rows;
  int32_t num_light_rows;
  int32_t num_split_rows;
  int32_t malformed;
  int32_t hash_error;        // hash accumulator: a table or count was inconsistent
  int32_t hash_split_rows;   // hash accumulator: rows that claimed a split slot (may exceed the capacity)
  int32_t hash_split_items;  // hash accumulator: chunks of the split rows
  int32_t pad1;
  int32_t hash_split_acc;    // hash accumulator: accumulator slots of the split rows
  int32_t hash_win_items;    // hash accumulator: output windows of the widest split rows
  int32_t hash_hist[64];     // hash accumulator: rows by floor(log2(products)), from kHashSplitMin up
  int64_t flops_total;
  int64_t nnz_total;
};

struct SplitRow {
  int32_t row, first, count, pad;
};

// Everything a row kernel needs about one TS-SpGEMM instance.
struct Problem {
  int32_t n;   // rows of A and B (A is n x n)
  int32_t d;   // columns of B and C
  int32_t wp;  // bitmap words per row
  const int32_t* arp;
  const int32_t* aci;
  const void* aval;
  const int32_t* brp;
  const int32_t* bci;
  const void* bval;
  const void* bcol;       // B's column ids narrowed to 8 (d <= 256) or 16 bits, for the numeric phase
  const uint32_t* bbits;  // B pattern, n x wp
  uint32_t* cbits;        // C pattern, n x wp
  int64_t* flops;         // per row
  const int2* ebnd;       // per A entry (brp[k], brp[k+1]) of its B row, or null: read by the
                          //   numeric staging instead of gathering B's row pointers
  int2* ebnd_w;           // or null: where the staging records the bounds it gathers
  const int32_t* crp;     // C row pointers
  int32_t* cci;
  void* cval;
};

struct SymParams {
  Problem pr;
  const Item* items;
  Counters* ctr;
  const uint32_t* mask;    // complement mask bitmap (n x wp) or null
  const uint32_t* active;  // wp words: columns that can still change, or null (all)
  const uint32_t* fnz;     // 1 bit per B row: row non-empty; null = no filter
  // Stop a row (or chunk) as soon as its accumulator holds every column the
  // mask leaves open among `active` ones: later B rows cannot change the
  // masked result. Only for pattern-only (OR, AND) work with a mask and fnz;
  // `flops` then counts the products examined, not all of them.
  bool early_exit;
  // rows with at most this many A entries are light: walked by the light-row
  // kernels, not listed (the same value as the binning's)
  int32_t light_max = kSlotRowMax;
};

// Item list layout: [split chunks][workgroup rows][wavefront rows][light rows].
struct NumParams {
  Problem pr;
  const Item* items;
  int32_t n_wg_items;       // split chunks + workgroup rows (one record per workgroup)
  int32_t n_heavy_records;  // + wavefront rows (one record per wavefront)
  int32_t n_light;          // light rows (one record per lane group)
  double* partial;          // split-chunk partial sums (slots x d), FP64
  int32_t* ipartial;        // same for the integer semiring
};

// ---------------------------------------------------------------- launchers
// All return TSSPGEMM_OK or an error code; all are asynchronous on `st`.
int launch_zero_bytes(void* p, size_t bytes, hipStream_t st);
int launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
// CSR pattern -> n x wp bitmap; with `narrow`, also the column ids as 1- or 2-byte values
int launch_csr_to_bitmap(int64_t n, const int32_t* rp, const int32_t* ci, int wp, uint32_t* bits, hipStream_t st,
                         void* narrow = nullptr, int narrow_bytes = 0);
int launch_nonempty_bits(int64_t n, const int32_t* rp, uint32_t* bits, hipStream_t st);
int launch_validate_csr(int64_t nrows, int64_t ncols, int64_t nnz, const int32_t* rp, const int32_t* ci,
                        Counters* ctr, hipStream_t st);

// zero_split: also clear the C bitmap row and product count of every split
// row (its chunks OR and add into them), in place of launch_sym_split_zero
// light_max: rows with at most this many A entries are light (not listed)
int launch_sym_bin(const Problem& pr, int32_t split_nnz, Item* items, Counters* ctr, hipStream_t st,
                   bool zero_split = false, int32_t light_max = kSlotRowMax);
int launch_symbolic(const SymParams& sp, int64_t max_items, hipStream_t st);
// The light-row kernel, the heavy-item kernel, or both (they touch disjoint
// rows, so they may run on two streams at once).
constexpr int kSymLight = 1, kSymHeavy = 2;
int launch_symbolic_part(const SymParams& sp, int64_t max_items, int part, hipStream_t st);
int launch_sym_split_zero(const Problem& pr, const Item* items, Counters* ctr, int64_t max_items, hipStream_t st);
int launch_sym_split_mask(const Problem& pr, const Item* items, const uint32_t* mask, Counters* ctr,
                          int64_t max_items, hipStream_t st);

// Work binning of the rows for the numeric phase (items in the layout of
// NumParams), done inside the count and row-pointer kernels of
// launch_count_scan: they walk the same rows.
struct NumBinArgs {
  NumThresholds th;
  Item* items;
  SplitRow* split_rows;
};
// popcount of each C bitmap row, exclusive scan -> c_rowptr, nnz(C) -> ctr;
// nb: null, or the numeric phase's binning of the same rows (by their
// product counts, set by the symbolic kernels)
int launch_count_scan(const Problem& pr, int32_t* cnt, int64_t* block_sums, int32_t* c_rowptr, Counters* ctr,
                      hipStream_t st, const NumBinArgs* nb = nullptr);
int64_t scan_block_sums_capacity(int64_t n);
int64_t exscan_workspace_bytes(int64_t n);
int launch_exscan_i32(const int32_t* in, int64_t n, int32_t* out, int64_t* block_sums, hipStream_t st);
int launch_exscan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* block_sums, hipStream_t st);



int launch_numeric(int sr, int group_lanes, int products, const NumParams& np, int64_t n_grid, hipStream_t st);
int col_id_bytes(int64_t d);  // 1 or 2: width of the narrowed column ids
int launch_split_finalize(int sr, const Problem& pr, const SplitRow* rows, int32_t nrows, const double* partial,
                          const int32_t* ipartial, hipStream_t st);
int launch_emit_pattern(const Problem& pr, hipStream_t st);

// Hash accumulator (d > kMaxDenseD, or chosen by tuning), d <= kHashMaxD.
constexpr int64_t kHashMaxD = 65536;
struct HashMask {
  const int32_t* rp;     // complement mask as CSR (sorted rows), or null
  const int32_t* ci;
  const uint32_t* bits;  // complement mask as bitmap rows of wpm words, or null
  int64_t wpm;
};
// Rows of a hash plan with many products are cut into chunks of A entries,
// each taken by its own workgroup: the symbolic phase ORs each chunk's
// columns into a global bitmap of the row, the numeric phase adds each
// product at the column's rank in that bitmap (a compact accumulator of the
// row's outputs).
struct HashSplit {
  int32_t* slot_of_row;  // n: the row's split slot, or -1
  int32_t* rows;         // cap: row of each slot
  int2* items;           // chunks: (slot, first A entry)
  uint32_t* bits;        // cap x words: the row's output columns
  int32_t* pref;         // cap x words: outputs of the row before each word
  int32_t* acc_off;      // cap: first accumulator of the row
  int2* wins;            // output windows of rows wider than a chunk's LDS array: (slot, window)
  int32_t* cls_rows;     // 4 x n: rows of each LDS table size class (outputs <= 64, 128, 256, 512)
  int32_t* cls_cnt;      // 6: rows in each table class, then chunks in each chunk class
  int32_t* chunk_lists;  // 2 x item_cap: chunks of rows with <= 1024 outputs, then of rows with more
  int32_t item_cap;      // capacity of the chunk list
  void* acc;             // accumulators (FP64, or INT32 for the integer semiring)
  int32_t cap;           // split slots (0: no row is split)
  int64_t split_flops;   // rows with at least this many products are split rows
  Counters* ctr;
};
// Products per row into pr.flops, and the histogram of floor(log2) of the
// products of rows with at least kHashSplitMin of them.
constexpr int64_t kHashSplitMin = 512;
int launch_hash_flops(const Problem& pr, int32_t* hist, hipStream_t st);
// From that histogram: the split threshold (a power of two >= kHashSplitMin
// whose rows' bitmaps fit the split budget) and the number of rows at or
// above it.
void hash_split_choose(const int32_t* hist, int64_t d, int64_t* split_flops, int64_t* rows);
int64_t hash_split_item_cap(int64_t a_nnz, int64_t cap);
int64_t hash_split_window_cap(int64_t cap, int64_t d);
// small_rows_only: every row that is not split has fewer than kHashSplitMin products
int launch_hash_symbolic(const Problem& pr, const HashMask& m, const HashSplit& hs, bool small_rows_only,
                         int32_t* cnt, int32_t* err, hipStream_t st);
int64_t hash_dense_workers(int64_t d);
// next: a device counter (4 bytes) for the long-row workers; split_rows,
// split_items and split_acc: the split counts the symbolic phase ended with;
// long_rows: some row that is not split may have more outputs than the LDS
// tables hold (else the long-row kernel is not launched)
// cls_n: rows of each table size class and chunks of each chunk class (the
// counts hs.cls_cnt ended with)
int launch_hash_numeric(int sr, const Problem& pr, const HashMask& m, const HashSplit& hs, int32_t split_rows,
                        int32_t split_items, int64_t split_acc, int32_t win_items, const int32_t* cls_n,
                        bool long_rows, void* strips, int32_t* err, int32_t* next, hipStream_t st);
// Rows at or above kHashSplitMin products in the histogram.
int64_t hash_split_candidates(const int32_t* hist);

}  // namespace tss
