/* tsspgemm.h -- C ABI of the TS-SpGEMM library for AMD Instinct MI355X (gfx950).
 *
 * TS-SpGEMM (Sec. II-A of "Distributed-Memory Parallel Algorithms for Sparse
 * Matrix and Sparse Tall-and-Skinny Matrix Multiplication", SC'24): C = A B
 * where A is a square n x n sparse matrix and B is a tall-and-skinny sparse
 * n x d matrix (d << n), over plus-times or over the Boolean (AND, OR)
 * semiring, the latter optionally with a complement mask (the multi-source
 * BFS step of Sec. IV-A, Algorithm 3). The local multiply is row-wise
 * Gustavson (Sec. III-A, Eq. 1) with a dense accumulator of width d for
 * d <= 1024 and a hash accumulator above (Sec. III-C), up to d = 65536.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer is a DEVICE pointer unless its comment says HOST.
 *  - The caller allocates every input and output buffer and keeps it alive
 *    until the work queued on `stream` has finished. The library owns only
 *    the workspace inside a plan / batch handle (freed by the matching
 *    *_destroy call) and a per-device scratch cache that the one-shot entry
 *    points (masked_bool, spmm, embed_epoch) reuse between calls. Calls on
 *    different streams that share it are ordered on the device (a call
 *    waits for the previous call when that one ran on another stream); work
 *    captured into a HIP graph is not, its replays are the caller's to order.
 *    Inputs are never modified.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is stream-ordered; only calls documented as "synchronizes" block
 *    the host (they return a count the caller needs to size an output).
 *  - CSR layout: rowptr[nrows+1] (rowptr[0] = 0, non-decreasing), colidx[nnz]
 *    strictly increasing within each row and in [0, ncols), int32; values in
 *    the order of colidx (float32 for PLUS_TIMES_F32, int32 for
 *    PLUS_TIMES_I32, unused and may be NULL for OR_AND). nnz must fit int32.
 *    With the environment variable TSSPGEMM_VALIDATE=1 inputs are checked on
 *    the device and TSSPGEMM_ERR_MALFORMED is returned for a broken one.
 *  - Return value: TSSPGEMM_OK (0) or a negative error code below. No C++
 *    exception crosses this boundary. tsspgemm_last_error() gives a message
 *    (thread-local) for the last failing call on this thread.
 */
#ifndef TSSPGEMM_H
#define TSSPGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSSPGEMM_OK 0
#define TSSPGEMM_ERR_INVALID_ARG (-1) /* null pointer, shape mismatch, bad enum   */
#define TSSPGEMM_ERR_MALFORMED (-2)   /* CSR invariant broken (validation on)     */
#define TSSPGEMM_ERR_OVERFLOW (-3)    /* nnz(C) or a row count exceeds INT32_MAX   */
#define TSSPGEMM_ERR_CAPACITY (-4)    /* caller's output too small; size returned  */
#define TSSPGEMM_ERR_UNSUPPORTED (-5) /* semiring / mask / size combination        */
#define TSSPGEMM_ERR_HIP (-6)         /* HIP runtime error (message kept)          */
#define TSSPGEMM_ERR_NOMEM (-7)       /* device workspace allocation failed        */

typedef struct {
  int64_t nrows, ncols, nnz;
  const int32_t* rowptr; /* nrows + 1 */
  const int32_t* colidx; /* nnz */
  const void* vals;      /* nnz values or NULL (pattern only) */
} tsspgemm_csr;

typedef enum {
  TSSPGEMM_PLUS_TIMES_F32 = 0, /* float inputs, FP64 accumulation, float output */
  TSSPGEMM_PLUS_TIMES_I32 = 1, /* int32, wrap-around (two's complement) sums     */
  TSSPGEMM_OR_AND = 2          /* pattern only: (AND, OR) semiring               */
} tsspgemm_semiring;

typedef enum {
  TSSPGEMM_MASK_NONE = 0,
  TSSPGEMM_MASK_COMPLEMENT_CSR = 1,   /* drop C(i,j) when (i,j) is stored in csr       */
  TSSPGEMM_MASK_COMPLEMENT_BITMAP = 2 /* drop C(i,j) when bit j of bits row i is set   */
} tsspgemm_mask_kind;

typedef struct {
  int32_t kind;            /* tsspgemm_mask_kind */
  const tsspgemm_csr* csr; /* n x d pattern (kind 1) */
  const uint32_t* bits;    /* n rows x tsspgemm_bitmap_words(d) words, bit j of row i at
                              word j/32, bit j%32 (kind 2) */
} tsspgemm_mask;

/* Accumulator of the numeric phase (Sec. III-C: a dense accumulator of
 * width d for d <= 1024, a hash accumulator above).
 *   LDS_STRIP:  lanes walk the entries of each B row and add into a d-wide
 *               strip in LDS (FP64 for the FP32 semiring). Needs d <= 1024.
 *   HASH:       for d > 1024. Short rows: an LDS open-addressing table of
 *               (column, sum) per row. Rows with many products: split into
 *               chunks of A entries over workgroups, with a global bitmap of
 *               the row's columns and sums at each column's rank in it. */
typedef enum {
  TSSPGEMM_ACC_AUTO = 0,
  TSSPGEMM_ACC_LDS_STRIP = 1,
  TSSPGEMM_ACC_HASH = 2
} tsspgemm_accumulator;

/* How the lanes of a group cover the products of the A entries they stage
 * (LDS strip accumulator).
 *   PER_B_ROW: each B row is read by group_lanes lanes, several rows in
 *              flight; lanes past a short row's end idle.
 *   FLAT:      the staged entries' products form one list (a scan of the B
 *              row lengths) and lane t takes products t, t + width, ...;
 *              pays when B rows are short next to the group width.
 *   VEC4:      as PER_B_ROW, but each lane reads four consecutive entries of
 *              the B row (4-aligned chunks: one 16-byte load of values, one
 *              load of column ids), so a wavefront keeps four times the B row
 *              bytes in flight per load instruction. Needs B's values 16-byte
 *              aligned in the numeric call; PER_B_ROW is used otherwise. */
typedef enum {
  TSSPGEMM_PRODUCTS_AUTO = 0,
  TSSPGEMM_PRODUCTS_PER_B_ROW = 1,
  TSSPGEMM_PRODUCTS_FLAT = 2,
  TSSPGEMM_PRODUCTS_VEC4 = 3
} tsspgemm_products;

/* Tuning knobs. A NULL tuning pointer, or a zero field, means "default".
 * The structure of C does not depend on any of these. Values are FP64 sums
 * rounded once to FP32 under every setting, each within the tolerance of the
 * exact sum; the settings add in different orders, so a value may in rare
 * cases round to a neighbouring FP32 under another setting. */
typedef struct {
  int32_t group_lanes;     /* lanes that stream one B row: 4,8,16,32,64 (0: from mean B row length) */
  int32_t wave_max_flops;  /* rows with at most this many products use one wavefront             */
  int32_t split_flops;     /* rows above this are split into chunks of about this many products   */
  int32_t sym_split_nnz;   /* symbolic pass: rows with more A entries than this are split (8192
                              unmasked with d <= 256, 16384 in the BFS, else 2048; a batch: 2048,
                              or its first tuning's)                                                */
  int32_t accumulator;     /* tsspgemm_accumulator: 0 auto, 1 LDS strip, 2 hash                    */
  int32_t light_max_flops; /* rows with at most this many products use one lane group            */
  int32_t products;        /* tsspgemm_products: how lanes cover a row's products                  */
} tsspgemm_tuning;

typedef struct tsspgemm_plan_s* tsspgemm_plan;

/* Number of 32-bit words per row of a bitmap of width d as used by this
 * library (d/32 rounded up to a power of two). */
int32_t tsspgemm_bitmap_words(int32_t d);

/* Symbolic phase (Sec. III-A, Eq. 1 structure; the symbolic nnz count of
 * Sec. III-D): computes flops per row (Sec. II-A), bins rows by work, the
 * output pattern (a d-bit bitmap per row for d <= 1024; per-row LDS hash
 * sets, or global bitmaps for split rows, with the hash accumulator) and C's
 * row pointers. With the hash accumulator it synchronizes `stream` twice
 * (once for the histogram of row products that sets the split rows).
 *   A: n x n, B: n x d (vals unused). sr: tsspgemm_semiring the plan is for.
 *   M: complement mask or NULL. tune: NULL for defaults.
 *   c_rowptr: caller-allocated, n + 1 int32, written.
 *   c_nnz: HOST out, nnz(C). Synchronizes `stream`.
 *   plan: in/out. If *plan is non-NULL its workspace is reused (grown as
 *   needed); otherwise a new plan is created. Destroy with tsspgemm_plan_destroy.
 *   With the hash accumulator the mask is copied into the plan (the numeric
 *   phase tests it again); the caller's mask may be freed after this call.
 * Errors: INVALID_ARG, UNSUPPORTED (d > 65536, or d > 1024 with the LDS strip
 * forced), OVERFLOW (nnz(C) > INT32_MAX), NOMEM, HIP. */
int tsspgemm_symbolic(const tsspgemm_csr* A, const tsspgemm_csr* B, int32_t sr, const tsspgemm_mask* M,
                      const tsspgemm_tuning* tune, int32_t* c_rowptr, int64_t* c_nnz, tsspgemm_plan* plan,
                      void* stream);

/* Numeric phase (Sec. III-A, Eq. 1 values; Sec. III-C accumulators): fills
 * C's column indices and values in the positions fixed by the plan. A and B
 * must have the patterns the plan was built with; their values may differ
 * between calls (so one plan serves every training step).
 *   c_colidx: nnz(C) int32, c_vals: nnz(C) float/int32 (NULL for OR_AND).
 * FP32 values are summed in FP64 and rounded once. With the LDS strip every
 * order of addition is fixed (results repeat bit for bit); the hash
 * accumulator adds with atomics in an order that may vary.
 * With the LDS strip and values, the plan's second numeric call records each
 * A entry's B row bounds (8 B per A entry of plan workspace, allocated by
 * that call), which later calls and tsspgemm_backward read instead of
 * gathering B's row pointers; a call being captured into a graph neither
 * records nor counts toward the second call.
 * Asynchronous. Errors: INVALID_ARG, NOMEM (the record's workspace), HIP. */
int tsspgemm_numeric(tsspgemm_plan plan, const tsspgemm_csr* A, const tsspgemm_csr* B, int32_t* c_colidx,
                     void* c_vals, void* stream);

/* Statistics of the last symbolic call on `plan` (HOST out pointers, any may
 * be NULL): total products (flops, Sec. II-A), nnz(C), and the number of
 * rows handled per lane group / per wavefront / per workgroup / split. For a
 * hash-accumulator plan only split_rows is set: the rows whose products are
 * cut into chunks of A entries taken by separate workgroups. */
int tsspgemm_plan_stats(tsspgemm_plan plan, int64_t* flops, int64_t* c_nnz, int64_t* light_rows,
                        int64_t* wave_rows, int64_t* block_rows, int64_t* split_rows);

void tsspgemm_plan_destroy(tsspgemm_plan plan);

/* One masked Boolean TS-SpGEMM (the N = A F, F = N \ S step of Algorithm 3,
 * Sec. IV-A): C = (A F over (AND, OR)) with the complement mask `visited`.
 *   F: n x d pattern. visited: mask (kind 1 or 2) or NULL.
 *   c_rowptr: n + 1 int32 (always written). c_colidx: capacity int32.
 *   c_nnz: HOST out. Synchronizes. If nnz(C) > c_capacity, returns
 *   TSSPGEMM_ERR_CAPACITY with *c_nnz and c_rowptr filled so the caller can
 *   grow and call again. */
int tsspgemm_masked_bool(const tsspgemm_csr* A, const tsspgemm_csr* F, const tsspgemm_mask* visited,
                         int32_t* c_rowptr, int32_t* c_colidx, int64_t c_capacity, int64_t* c_nnz, void* stream);

/* Multi-source BFS (Sec. IV-A, Algorithm 3) from d sources by repeated masked
 * Boolean TS-SpGEMM until every frontier is empty. Vertex i is reached from
 * k when A(i,k) != 0 (the product A F).
 *   A: n x n pattern. sources: d vertex ids in [0, n) (device).
 *   levels: n x d int32 row-major, fully written: level[v*d + s] = BFS depth
 *   of v from sources[s] (0 at the source, -1 if unreachable).
 *   iterations: HOST out, number of masked products performed (the last one
 *   yields the empty frontier).
 *   frontier_nnz: HOST array of `capacity` int64 or NULL: nnz(F) after each
 *   product (the last entry is 0).
 *   Synchronizes once per iteration. 1 <= d <= 1024. A source outside
 *   [0, n) gives TSSPGEMM_ERR_INVALID_ARG. Device memory: one n x d bitmap per
 *   iteration plus two more, and O(n) workspace, kept per device between
 *   calls (grown as needed); calls on one device are serialized, and a call
 *   on another stream waits on the device for the previous one. */
int tsspgemm_msbfs(const tsspgemm_csr* A, const int32_t* sources, int32_t d, int32_t* levels, int32_t* iterations,
                   int64_t* frontier_nnz, int32_t capacity, void* stream);

/* CSR transpose of A's pattern (the single-GPU form of the column-partitioned
 * copy A^c of Sec. III-A): at_rowptr (ncols+1), at_colidx (nnz) with rows
 * listed in ascending order, at_perm (nnz): position in A of each entry.
 * Allocates temporaries (four nnz-sized key/value buffers of the radix sort)
 * and synchronizes `stream` before freeing them: meant to run once per
 * pattern, outside timed or captured loops. Errors: INVALID_ARG, NOMEM, HIP. */
int tsspgemm_transpose(const tsspgemm_csr* A, int32_t* at_rowptr, int32_t* at_colidx, int32_t* at_perm,
                       void* stream);

/* Backward of a plus-times TS-SpGEMM for a loss L with G = dL/dC given on
 * C's pattern (G->rowptr/colidx equal C's, G->vals float):
 *   grad_a[p] = sum over j in pat(B_k) of G(i,j) B(k,j) for the p-th entry
 *   (i,k) of A (an SDDMM on A's pattern);
 *   grad_b[q] = sum over i with (i,k) in pat(A) of A(i,k) G(i,j) for the q-th
 *   entry (k,j) of B (A^T G sampled on B's pattern), using A^T from
 *   tsspgemm_transpose.
 * plan: the forward plus-times FP32 plan of C = A B, required: its binned
 * rows drive grad_a (G's row i is staged in LDS, so every G(i,j) the row's
 * products need is read from there). Sums are FP64 in a fixed order,
 * rounded once to FP32 (reproducible). grad_b runs the two passes of
 * tsspgemm_backward below (same workspace, same single synchronization at
 * its first call on a plan); grad_a alone is asynchronous.
 * Errors: INVALID_ARG (NULL plan or output, a plan of another semiring or
 * built with a mask, A / B / G / AT not matching the plan), UNSUPPORTED (a
 * hash-accumulator plan), NOMEM, HIP. */
int tsspgemm_grad_a(tsspgemm_plan plan, const tsspgemm_csr* A, const tsspgemm_csr* B, const tsspgemm_csr* G,
                    float* grad_a, void* stream);
int tsspgemm_grad_b(tsspgemm_plan plan, const tsspgemm_csr* AT, const int32_t* at_perm, const tsspgemm_csr* A,
                    const tsspgemm_csr* B, const tsspgemm_csr* G, float* grad_b, void* stream);

/* Both gradients of the same backward in one call (either output may be
 * NULL, not both; AT / at_perm are needed when grad_b is requested). One
 * pass over A's rows (the forward plan's binned rows, G's row i in an LDS
 * strip) forms the dL/dA dot products and writes the G(i, j) each product
 * (i,k) x (k,j) reads, in one block per A entry; a second pass walks A^T and
 * sums A(i,k) G(i,j) from those blocks for each entry (k, j) of B. Values
 * equal those of tsspgemm_grad_a and tsspgemm_grad_b (same sums in the same
 * order), which run the same passes. The block of entry (i,k) holds
 * A(i,k) and then G(i,j) for j in pat(B_k), padded to a multiple of 64
 * bytes; blocks are stored in A^T order, so the second pass reads each B
 * row's blocks contiguously. Workspace in the plan, allocated at the first
 * call and kept: the blocks (4 bytes per product of the forward plus at most
 * 64 bytes per A entry), 4 bytes per A entry (its block's place), 16 bytes
 * per row, and the dL/dB work list. The first call on a plan that asks for
 * grad_b builds the blocks' starts and synchronizes `stream` once (to size
 * the buffer); later calls are asynchronous. Errors as tsspgemm_grad_b. */
int tsspgemm_backward(tsspgemm_plan plan, const tsspgemm_csr* AT, const int32_t* at_perm, const tsspgemm_csr* A,
                      const tsspgemm_csr* B, const tsspgemm_csr* G, float* grad_a, float* grad_b, void* stream);

/* Sparse times dense tall-and-skinny (SpMM), the alternative Sec. V-C
 * compares TS-SpGEMM with: C = A B with B and C dense, plus-times over FP32,
 * FP64 sums in a fixed order rounded once to FP32.
 *   A: n x n CSR with float values. B: n rows of d floats, row-major with
 *   leading dimension ldb >= d (zeros included). C: n x d, leading dimension
 *   ldc >= d, every entry written (rows of A without entries give 0).
 *   1 <= d <= 1024 (d = 0 or n = 0: nothing to do).
 * Uses the device's workspace cache (calls on different streams are
 * ordered on the device, see the conventions above). Asynchronous.
 * Errors: INVALID_ARG, UNSUPPORTED (d > 1024), NOMEM, HIP. */
int tsspgemm_spmm(const tsspgemm_csr* A, const float* B, int64_t d, int64_t ldb, float* C, int64_t ldc,
                  void* stream);

/* The same SpMM for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * arguments, result and summation order are those of tsspgemm_spmm (the
 * same kernels), but the workspace (counters, chunk list, long-row records,
 * FP64 partial rows) lives in a fixed device array of the library of
 * TSSPGEMM_SPMM_NOALLOC_MAX_BYTES per GPU, held from the first use on that
 * GPU until the process ends. No hipMalloc, hipFree or allocating call is
 * made. The workspace bound is about nnz(A) * d / 8 bytes
 * (256 + (2 nnz/128 + 1) * (8 + 8 d) + (nnz/128 + 1) * 16, each part rounded
 * up to 256 bytes); a larger problem returns TSSPGEMM_ERR_CAPACITY, with the
 * bytes it would need in the message. Every call on one GPU shares that
 * GPU's array (its counters are cleared by a kernel at the start of each
 * call): calls that overlap on one GPU, on any streams, race.
 * Asynchronous. Errors: INVALID_ARG, UNSUPPORTED (d > 1024), CAPACITY, HIP. */
#define TSSPGEMM_SPMM_NOALLOC_MAX_BYTES (64ll << 20)
int tsspgemm_spmm_noalloc(const tsspgemm_csr* A, const float* B, int64_t d, int64_t ldb, float* C, int64_t ldc,
                          void* stream);

/* One pass of the sparse force-directed embedding update (Sec. IV-B) over
 * rows [row_begin, row_end) of Z, in minibatches of batch_rows rows taken in
 * row order (the minibatch is the tile height of Sec. IV-B).
 *   A: n x n CSR with float values: > 0 a neighbour (attractive), < 0 a
 *      negative sample (repulsive), 0 no force. Sorted columns.
 *   Z: n x d embedding with exactly k entries per row, row i at i * k in
 *      z_colidx (ascending, distinct columns < d) and z_vals (float). Updated
 *      in place for the rows in range; other rows are read only.
 * For each row i of a minibatch, reading Z as it was when the minibatch
 * started: s = z_i . z_j, sig = 1 / (1 + exp(-s)), F_i = sum over stored
 * (i, j, a) of w z_j with w = 1 - sig (a > 0), -sig (a < 0); u = z_i + lr F_i
 * in FP64, rounded once to float; the new row holds the k entries of largest
 * |u| (ties: lower column), sorted by column.
 * 1 <= k <= d <= 1024, batch_rows >= 1, 0 <= row_begin <= row_end <= n.
 * Uses the device's workspace cache (a second n x k copy of Z, per-row
 * counters, partial forces of long rows; calls on different streams are
 * ordered on the device, see the conventions above). Asynchronous; no
 * allocation after the first call of a given size
 * (n, nnz(A), d, and whether batch_rows <= 4096: such minibatches cut long
 * rows into shorter chunks, with a larger partial-force buffer).
 * Errors: INVALID_ARG, UNSUPPORTED (d > 1024), NOMEM, HIP. */
int tsspgemm_embed_epoch(const tsspgemm_csr* A, int64_t d, int64_t k, int32_t* z_colidx, float* z_vals, float lr,
                         int64_t batch_rows, int64_t row_begin, int64_t row_end, void* stream);

/* Column tile of A (Sec. III-B): A(:, c0:c1), every row, column ids kept, so
 * that (A(:, c0:c1)) B reads only B's rows c0..c1-1. Two calls: the count
 * fills out_rowptr (nrows + 1, device) and writes the tile's nnz to *out_nnz
 * (HOST; synchronizes once); the fill writes out_colidx / out_vals (nnz
 * entries; out_vals may be NULL for the pattern only). 0 <= c0 <= c1.
 * Both allocate temporaries. Errors: INVALID_ARG, NOMEM, HIP. */
int tsspgemm_column_slice_count(const tsspgemm_csr* A, int32_t c0, int32_t c1, int32_t* out_rowptr,
                                int64_t* out_nnz, void* stream);
int tsspgemm_column_slice_fill(const tsspgemm_csr* A, int32_t c0, int32_t c1, const int32_t* out_rowptr,
                               int32_t* out_colidx, float* out_vals, void* stream);

/* Merge of partial outputs (Algorithm 2, Merge; Sec. III-C: a dense
 * accumulator for small d): C = sum of `count` n x d CSR parts (parts is a
 * HOST array of descriptors; sorted columns; float values). Output pattern:
 * the union of the parts' patterns; values: FP64 sums with the parts added in
 * order, rounded once. 1 <= count <= 64, d <= 1024. The count writes
 * out_rowptr (n + 1) and *out_nnz (HOST; synchronizes once; allocates
 * temporaries); the values call writes out_colidx / out_vals (asynchronous).
 * Errors: INVALID_ARG, UNSUPPORTED (count > 64 or d > 1024), NOMEM, HIP. */
int tsspgemm_merge_count(int32_t count, const tsspgemm_csr* parts, int32_t* out_rowptr, int64_t* out_nnz,
                         void* stream);
int tsspgemm_merge_values(int32_t count, const tsspgemm_csr* parts, const int32_t* out_rowptr, int32_t* out_colidx,
                          float* out_vals, void* stream);

/* Batched plus-times TS-SpGEMM: `count` independent instances C_t = A_t B_t
 * (FP32 values, d_t <= 1024): every symbolic phase one launch over all
 * instances, the work of all instances binned into one list (by instance,
 * heaviest first); the numeric phase one pair of launches per class of
 * instances with the same group widths, product layout and LDS strip size.
 * tsspgemm_batched_plan sizes everything once (it runs the symbolic phase;
 * synchronizes); the patterns of A_t and B_t must not change afterwards,
 * their values may. The plan also records each A entry's B row bounds (8 B
 * per A entry of batch workspace), which the numeric phase reads.
 *   As, Bs: HOST arrays of `count` descriptors (device data).
 *   tune: NULL (one group width and product layout for the whole batch,
 *   from the mean B row length over all instances), or a HOST array of
 *   `count` tunings, each instance's own (except sym_split_nnz, the
 *   batch's: the first tuning's).
 *   pool_capacity: HOST out, sum of nnz(C_t) = entries of the output pool.
 *   rowptr_total: HOST out, sum of (n_t + 1).
 * tsspgemm_batched_run queues the whole batch (symbolic, scans, numeric) on
 * `stream` with no host synchronisation and no allocation (so it can be
 * captured in a HIP graph):
 *   c_rowptrs: rowptr_total int32; instance t's row pointers start at
 *   sum_{s<t} (n_s + 1) and are relative to its own output.
 *   pool_colidx / pool_vals: pool_capacity entries.
 *   c_offsets: count + 1 int64 (device); instance t's output occupies
 *   [c_offsets[t], c_offsets[t+1]) of the pool.
 * tsspgemm_batched_capture records that same run into a HIP graph kept in the
 * batch (the output arrays are fixed at capture time) and
 * tsspgemm_batched_launch replays it on `stream`.
 * tsspgemm_batched_flops copies the products of each instance (count int64,
 * HOST) from the last completed run or plan. */
typedef struct tsspgemm_batch_s* tsspgemm_batch;
int tsspgemm_batched_plan(int32_t count, const tsspgemm_csr* As, const tsspgemm_csr* Bs,
                          const tsspgemm_tuning* tune, tsspgemm_batch* out, int64_t* pool_capacity,
                          int64_t* rowptr_total, void* stream);
int tsspgemm_batched_run(tsspgemm_batch batch, int32_t* c_rowptrs, int32_t* pool_colidx, float* pool_vals,
                         int64_t* c_offsets, void* stream);
int tsspgemm_batched_capture(tsspgemm_batch batch, int32_t* c_rowptrs, int32_t* pool_colidx, float* pool_vals,
                             int64_t* c_offsets);
int tsspgemm_batched_launch(tsspgemm_batch batch, void* stream);
int tsspgemm_batched_flops(tsspgemm_batch batch, int64_t* flops);
void tsspgemm_batched_destroy(tsspgemm_batch batch);

/* Message for the last failing call on this thread ("" if none). */
const char* tsspgemm_last_error(void);

/* Library version string. */
const char* tsspgemm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TSSPGEMM_H */
