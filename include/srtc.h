/*
 * srtc -- semiring sparse tensor contraction on AMD MI355X (gfx950).
 *
 * C-ABI of the library libsrtc.so.  The operation is the generalized tensor
 * contraction of Solomonik and Hoefler, "Sparse Tensor Algebra as a Parallel
 * Programming Model" (arXiv:1512.00066):
 *
 *     C["c"] (+)= A["a"] (x) B["b"]
 *
 * over a semiring ((+), additive identity, (x)) chosen by the caller
 * (Section 3.1, Table 1), with operands given by index strings in Einstein
 * notation (Section 3.3.1): an index in A and B but not C is contracted, an
 * index in A (or B) and C is a free row (column) index, an index in all three
 * tensors enumerates independent problems.  Every contraction is folded to a
 * matrix product first (Section 5.1): rows = free indices of A, inner =
 * contracted indices, columns = free indices of B.  Contracting two sparse
 * tensors, and producing sparse output, are the extensions the paper leaves
 * open (Sections 1 and 7); this library computes both.
 *
 * Conventions for every call:
 *   - Pointers inside srtc_tensor are DEVICE pointers unless stated; host
 *     pointers are marked "host".
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Work is enqueued on it; calls that must know an output size
 *     synchronize that stream once (documented per call).
 *   - Inputs are borrowed: they must stay valid until the stream work ends.
 *   - Device memory comes from the context's allocator callback (outputs,
 *     which become the caller's, and scratch, returned through the free
 *     callback before the call ends).  The allocator must be stream-ordered
 *     (a caching allocator bound to `stream`, as torch's is) or synchronous.
 *     Without a callback, outputs come from hipMalloc and scratch from a
 *     per-context cache of hipMalloc blocks kept until srtc_ctx_destroy.
 *   - Environment (read by srtc_ctx_create):
 *       SRTC_TRACE=1          prints each phase of every call to stderr;
 *       SRTC_VALIDATE=1       checks every sparse operand's structure as
 *                             opts.validate does (SRTC_ERR_FORMAT);
 *       SRTC_FORCE_SCHEDULE=k SpGEMM schedule k (0..SRTC_NUM_SCHEDULES-1)
 *                             wherever the caller leaves the choice open
 *                             (opts.schedule = -1);
 *       SRTC_LDS_BUDGET=bytes LDS per workgroup the SpGEMM kernels may use:
 *                             rows whose kernel would need more go to
 *                             narrower dense windows (more passes, the same
 *                             results); SRTC_ERR_UNSUPPORTED if even the
 *                             narrowest window does not fit.
 *       SRTC_HUB_TILE=k       opts.hub_tile for calls that leave it 0
 *                             (1..16384);
 *       SRTC_COL_BLOCKS=q     multiply the rows with many products one
 *                             column block of B at a time (q >= 2 blocks; 0:
 *                             blocks of about 48 MB of B); unset or 1: no
 *                             blocks.  The results are the same.
 *     srtc_ctx_create returns SRTC_ERR_ARG for a malformed value.
 *   - No call aborts and no C++ exception crosses the ABI: failures return a
 *     negative srtc_status and srtc_last_error() describes the last one.
 *   - An operand entry equal to the additive identity is absent; output
 *     entries equal to it are dropped (a new sparse tensor holds no entries,
 *     a dense one holds the additive identity: Section 3.2).
 */
#ifndef SRTC_H
#define SRTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- statuses -- */
typedef enum srtc_status {
  SRTC_OK = 0,
  SRTC_ERR_ARG = -1,           /* null pointer, negative size, bad enum value */
  SRTC_ERR_INDEX = -2,         /* bad index string: length, repeated index,
                                  index in only one tensor (reductions and maps
                                  of Section 3.3.1 are not part of this API) */
  SRTC_ERR_DIM = -3,           /* dimensions of matched indices differ */
  SRTC_ERR_DTYPE = -4,         /* value type not defined for the semiring */
  SRTC_ERR_FORMAT = -5,        /* malformed CSR/COO (checked when validate=1) */
  SRTC_ERR_ALIAS = -6,         /* output storage overlaps an input */
  SRTC_ERR_OOM = -7,           /* the allocator returned NULL */
  SRTC_ERR_NOT_CONVERGED = -8, /* fixpoint still changing after max_iters */
  SRTC_ERR_UNSUPPORTED = -9,   /* well-formed request outside this library */
  SRTC_ERR_DEVICE = -10,       /* HIP runtime error (message has the text) */
  SRTC_ERR_TOO_LARGE = -11     /* request exceeds a fixed-size buffer
                                  (srtc_contract_noalloc) */
} srtc_status;

/* ------------------------------------------------------------ semirings -- */
/* Section 3.1: a semiring is (additive op, additive identity, multiplicative
 * op, multiplicative identity).  The additive identity is passed by the
 * caller (add_id, a host pointer to one value of the operand dtype; NULL
 * selects the default listed here). */
typedef enum srtc_semiring {
  SRTC_PLUS_TIMES = 0, /* (+, 0, x, 1) on F64/F32.  add_id must be 0.  F32
                          with a sparse operand: products are formed exactly
                          in fp64 and summed in fp64, rounded once (relative
                          error <= 2^-24 + t 2^-53 for t non-negative terms).
                          F32 dense x dense on the matrix cores: fp32
                          multiply-adds sum at most 128 consecutive k-terms
                          in fp32, each partial sum then added into an fp64
                          total, so |error| <= 128 * 2^-24 * sum_k |a_ik
                          b_kj| (relative <= 7.7e-6 for non-negative data;
                          signed data can cancel, and the bound is then on
                          the sum of magnitudes, not on |c|). */
  SRTC_MIN_PLUS = 1,   /* tropical (min, id, +, 0) on I32 (default id
                          INT32_MAX/2, Section 3.1; id must lie in
                          1..INT32_MAX/2, SRTC_ERR_ARG otherwise) or F32
                          (default +inf).  I32 operands must lie in [-id, id]
                          (checked with validate), so no sum overflows; a
                          result at or above id is absent: dropped from a
                          sparse output, stored as id in a dense one. */
  SRTC_OR_AND = 2,     /* boolean (or, false, and, true) on BOOL8 (any nonzero
                          byte is true) and BITS64 frontiers */
  SRTC_MAX_TIMES = 3   /* (max, id, x, 1) on F32/F64; default id 0 (for
                          non-negative values) */
} srtc_semiring;

typedef enum srtc_dtype {
  SRTC_F64 = 0,
  SRTC_F32 = 1,
  SRTC_I32 = 2,
  SRTC_BOOL8 = 3,  /* uint8 0/1 */
  SRTC_BITS64 = 4, /* dense boolean frontier: bit s of word v = source s */
  SRTC_PATH64 = 5  /* a path as one uint64: weight (bits 32..63, >= 0) and
                      hop count (bits 0..31); with MIN_PLUS the additive op
                      keeps the lighter path, the one with fewer hops on a
                      tie, and the product adds weights and hops (the
                      hop-carrying tropical semiring of Section 4.2's path
                      doubling); identity = weight INT32_MAX/2, 0 hops */
} srtc_dtype;

typedef enum srtc_format {
  SRTC_DENSE = 0, /* row-major, last mode fastest, prod(dims) values */
  SRTC_COO = 1,   /* nnz index-value pairs: coo_keys[t] = linearized index
                     (last mode fastest), vals[t]; duplicates allowed (they
                     are combined with the additive op) */
  SRTC_CSR = 2    /* rows = leading `split` modes, columns = the rest;
                     rowptr[rows+1] int64, colidx[nnz] int32 ascending and
                     unique within a row, vals[nnz] */
} srtc_format;

#define SRTC_MAX_ORDER 8

typedef struct srtc_tensor {
  int32_t order;                 /* 0..SRTC_MAX_ORDER */
  int32_t format;                /* srtc_format */
  int32_t dtype;                 /* srtc_dtype */
  int32_t split;                 /* CSR: number of leading modes in the row */
  int64_t dims[SRTC_MAX_ORDER];  /* extent of each mode */
  int64_t nnz;                   /* COO/CSR: stored entries */
  int64_t *coo_keys;             /* COO */
  int64_t *rowptr;               /* CSR */
  int32_t *colidx;               /* CSR */
  void *vals;                    /* COO/CSR: nnz values; DENSE: prod(dims) */
} srtc_tensor;

/* Allocator callback: return `bytes` of device memory (256-byte aligned) or
 * NULL.  Free callback: release a pointer returned by the allocator. */
typedef void *(*srtc_alloc_fn)(void *user, size_t bytes);
typedef void (*srtc_free_fn)(void *user, void *ptr);

typedef struct srtc_ctx srtc_ctx;

/* Number of SpGEMM schedules (the variant/binning presets the autotuner and
 * the selector choose among); a schedule is named by its index. */
#define SRTC_NUM_SCHEDULES 8
typedef int32_t srtc_schedule; /* 0..SRTC_NUM_SCHEDULES-1 */
#define SRTC_NUM_FEATURES 32

typedef struct srtc_opts {
  int32_t schedule; /* -1: choose (selector if trained, else autotune cache,
                       else the default); 0..SRTC_NUM_SCHEDULES-1: force */
  int32_t sorted;   /* 1: output rows list columns ascending (default) */
  int32_t validate; /* 1: check operand structure (SRTC_ERR_FORMAT) */
  int32_t hub_tile; /* > 0 (at most 16384): sparse x sparse (+,x) products
                       on F64/F32 form the block of the hub_tile rows of A,
                       inner indices and columns of B with the most entries
                       as one dense product on the matrix cores (Section 6.2's
                       small dense blocks, see srtc_contract); 0: the
                       environment's SRTC_HUB_TILE, else none */
} srtc_opts;

/* ------------------------------------------------------------- context -- */

/* Create a context bound to HIP device `device`.  alloc/free may be NULL:
 * then hipMalloc/hipFree are used (synchronous).  One context per host
 * thread. */
srtc_status srtc_ctx_create(int device, srtc_alloc_fn alloc, srtc_free_fn free_fn, void *user,
                            srtc_ctx **out);
srtc_status srtc_ctx_destroy(srtc_ctx *ctx);
/* Message for the last failed call on this context (never NULL). */
const char *srtc_last_error(const srtc_ctx *ctx);
const char *srtc_status_string(srtc_status st);

/* ------------------------------------------------------------ profile -- */

/* Per-kernel profile (for measuring a kernel against its roofline).  While
 * enabled, every kernel launch outside graph capture is bracketed by HIP
 * events recorded on the stream it runs on, and the launch's algorithmic
 * byte count (what the operation must read and write, not what the cache
 * hierarchy moves) is added to its entry.  Enabling clears the table. */
srtc_status srtc_profile_enable(srtc_ctx *ctx, int32_t on);
/* Entry idx (0-based; SRTC_ERR_ARG past the end): kernel name (copied into
 * name[name_len], host), launches, total milliseconds and total algorithmic
 * bytes.  Waits for the recorded events. */
srtc_status srtc_profile_query(srtc_ctx *ctx, int32_t idx, char *name, int32_t name_len, int64_t *launches,
                               double *total_ms, double *total_bytes);

/* ---------------------------------------------------------------- fold -- */

/* Fold (Section 5.1, local transposition of Section 6.2): rearrange a COO or
 * CSR tensor `src`, whose modes carry the letters of `isrc`, into a CSR
 * matrix whose row key linearizes the modes named by `rows` (in that order)
 * and whose column key linearizes those named by `cols`.  Every letter of
 * isrc must appear exactly once in rows+cols.  Duplicate keys are combined
 * with the semiring's additive op in input order (float (+) in fp64, rounded
 * once), identity entries are dropped.  A CSR source is transposed this way.
 * On success `out` is a CSR tensor of order |rows|+|cols| with
 * split = |rows|; its arrays come from the allocator and belong to the
 * caller.  Synchronizes `stream` once (output size). */
srtc_status srtc_fold(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, const char *isrc,
                      const srtc_tensor *src, const char *rows, const char *cols,
                      srtc_tensor *out, void *stream);

/* ----------------------------------------------------------- contract -- */

/* C["ic"] (+)= A["ia"] (x) B["ib"] (Section 3.3.1; accumulate = 0 gives
 * C = A (x) B).  Forms:
 *   sparse A x sparse B -> sparse C (CSR, allocated here; with accumulate the
 *       previous C joins the sum and is replaced by new arrays -- the old
 *       arrays stay the caller's: each row's accumulator starts from the old
 *       row's entries, as one more term of the sum, unless C interleaves its
 *       letters or has a letter in all three tensors, where the product is
 *       merged into the old C afterwards).  Synchronizes a few times (bin
 *       and output sizes).
 *   sparse A x dense B  -> dense C (caller-allocated, fully asynchronous).
 *   dense A x dense B   -> dense C, (+,x) only, on the matrix cores (a
 *       letter in all three tensors makes it a strided batch of GEMMs);
 *       when every letter is in all three tensors, the elementwise
 *       product, for any semiring.
 * Index rules: each letter appears at most once per tensor and in at least
 * two tensors.  Letters may come in any order in every tensor (Section
 * 5.1's folding): operands are folded or permuted to (rows, inner) and
 * (inner, columns) form, and when C's order interleaves its row letters
 * (those of A) with its column letters (those of B only) the product is
 * formed in (rows, columns) order and folded back into C's order (a dense
 * permutation through scratch of C's size; for a sparse C a re-fold whose
 * CSR rows are C's first |row letters| letters).  Sparse operands may be
 * COO (folded on the fly) or CSR whose split matches the fold.
 * Right-hand sides are read before C is written (out-of-place); C may not
 * share storage with A or B (SRTC_ERR_ALIAS).
 * Hub tiles (opts->hub_tile = k > 0, (+,x) on F64/F32, sparse x sparse, no
 * letter in all three tensors, no old C entries to merge): H_i, H_k, H_j are
 * the k rows of A, inner indices and columns of B with the most entries
 * (A's row lengths; A's column counts plus B's row lengths; B's column
 * counts; ties to the smaller index).  D = A[H_i,H_k] B[H_k,H_j] is formed
 * densely on the matrix cores (F32: fp32 multiply-adds of at most 128 terms
 * each added into fp64, as for dense x dense) and the rest sparsely, as one
 * product [A_x | A_h | I] x [B ; B_x ; D] (A_h = A's entries in H_i x H_k,
 * A_x the others, B_x = B's rows in H_k without the H_j columns).  The
 * pattern of C is the same; values differ from the sparse path only by
 * summation order (and, for F32, the tile's rounding). */
srtc_status srtc_contract(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, int accumulate,
                          const char *ia, const srtc_tensor *A, const char *ib,
                          const srtc_tensor *B, const char *ic, srtc_tensor *C,
                          const srtc_opts *opts, void *stream);

/* srtc_contract's sparse x dense -> dense form for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): no allocator callback, hipMalloc,
 * hipFree or allocating library routine is called.  The work-item plan and
 * the partial results of long rows live in one fixed device buffer of the
 * library (64 MiB per device, looked up when a context is created and kept
 * until the process ends).  Arguments and results as srtc_contract with
 * opts = NULL, restricted to the layouts that need no rearrangement:
 *   A  CSR; ia = C's row letters (in C's order) then the contracted
 *      letters; split = number of row letters;
 *   B  dense; ib = the contracted letters in A's order, then C's column
 *      letters in C's order;
 *   C  dense, caller-allocated; ic = row letters then column letters;
 *   no letter in all three tensors.
 * Any other layout: SRTC_ERR_UNSUPPORTED.  The plan takes about
 *   40 m + 32 (m + nnz/T) + 16 (nnz/T) s
 * bytes (m rows of A, s columns of C, T = 32..256 nonzeros per work item);
 * a product needing more than the buffer returns SRTC_ERR_TOO_LARGE.
 * SRTC_VALIDATE is not applied here (validation allocates), and the call
 * leaves no srtc_profile record (it takes no HIP events).  Fully
 * asynchronous.  Every call on a device shares that device's buffer and
 * leaves its contents behind; calls that overlap on one device (two
 * streams, two threads or two contexts) race and must be ordered by the
 * caller. */
srtc_status srtc_contract_noalloc(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, int accumulate,
                                  const char *ia, const srtc_tensor *A, const char *ib, const srtc_tensor *B,
                                  const char *ic, srtc_tensor *C, void *stream);

/* Contraction into a given output pattern (the output with predefined
 * sparsity that Sections 1 and 7 name as an extension):
 *   C[ic] = M (.) (A[ia] (x) B[ib])
 * Only positions present in the mask M (same index string and extents as C;
 * COO or CSR; its values are ignored, duplicates merge) are formed; every
 * product landing elsewhere is dropped.  A and B are sparse (COO or CSR);
 * no index may appear in all of A, B and C.  C (host descriptor, device
 * buffers from the allocator) receives a CSR over C's row letters whose
 * pattern is a subset of M's: positions with no product, or whose result is
 * the additive identity, are absent; rows list columns in ascending order.
 * opts: only `validate` is used (checks A, B and M).  One host sync. */
srtc_status srtc_contract_masked(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, const char *ia,
                                 const srtc_tensor *A, const char *ib, const srtc_tensor *B, const char *ic,
                                 const srtc_tensor *M, srtc_tensor *C, const srtc_opts *opts, void *stream);

/* Consumer of one row panel of a streamed product (srtc_contract_panels).
 * C_panel is a CSR matrix (order 2, split 1) holding rows [row0, row0 +
 * nrows) of C folded to a matrix (rows: C's row letters linearized, columns:
 * its column letters), with row pointers relative to the panel
 * (rowptr[0] = 0).  Its three arrays come from the context's allocator and
 * are the consumer's to keep or release; the work that forms them is on
 * `stream`, so device work the consumer enqueues there sees them.  Return 0
 * to continue; nonzero stops the product. */
typedef int32_t (*srtc_panel_fn)(void *user, int64_t row0, int64_t nrows, srtc_tensor *C_panel,
                                 void *stream);

/* C[ic] = A[ia] (x) B[ib] for sparse A and B, formed and handed over one
 * row panel at a time, for outputs larger than the device memory (the
 * paper maps contractions under a memory constraint, Section 5.1; one GPU
 * streams the output instead of replicating it).  Panels are consecutive
 * runs of C's rows cut so that each holds at most `panel_products` products
 * (<= 0: 2^31), a row with more forming a panel alone; a panel has at most
 * as many entries as products.  Operands are folded once and the schedule is
 * chosen once for the whole product (opts->schedule, or as srtc_contract
 * chooses from the features of all rows); every panel is one SpGEMM of its
 * rows of A with all of B, then `consume` receives it.  Tables built from B
 * alone (its window tables and value records) are built for the first panel
 * and reused by the others, so A and B must not change until the call
 * returns (the consumer may not write them).  Rules as
 * srtc_contract, except: no letter in all three tensors, and C lists its
 * row letters first.  SRTC_ERR_ARG if the consumer stops the product (the
 * panels handed over so far stay the consumer's).  Synchronizes a few times
 * per panel. */
srtc_status srtc_contract_panels(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, const char *ia,
                                 const srtc_tensor *A, const char *ib, const srtc_tensor *B, const char *ic,
                                 const srtc_opts *opts, int64_t panel_products, srtc_panel_fn consume,
                                 void *user, void *stream);

/* ----------------------------------------------------------- fixpoint -- */

/* Bellman-Ford as repeated semiring products (Section 4.2):
 *   X <- X (+) A (x) X
 * on a dense n x s frontier X (row-major, updated in place) until a step
 * changes nothing.  A is an n x n CSR whose entry (i, j) is the weight of
 * edge j -> i.  Steps are replayed as captured HIP graphs of
 * `steps_per_check` steps; the host reads the change flags once per replay.
 * *iters_out (host) = number of steps up to and including the first
 * unchanged one.  Returns SRTC_ERR_NOT_CONVERGED if step `max_iters` (<= 0:
 * n) still changed something (a negative cycle, for (min,+)); X then holds
 * that iterate.  Supported: MIN_PLUS (I32, F32), MAX_TIMES (F32, F64),
 * OR_AND (BOOL8). */
srtc_status srtc_fixpoint(srtc_ctx *ctx, srtc_semiring sr, const void *add_id,
                          const srtc_tensor *A, srtc_tensor *X, int64_t max_iters,
                          int32_t steps_per_check, int64_t *iters_out, void *stream);

/* srtc_fixpoint with options.  flags:
 *   SRTC_FIXPOINT_CHANGED_ROWS  each step gathers only from rows of X that
 *     changed in the previous step (the first step from all rows).  An
 *     unchanged row's term is already part of every row it reaches, and the
 *     additive op of every supported semiring is idempotent, so the
 *     iterates, X and *iters_out are exactly those of srtc_fixpoint; the
 *     gathers drop to the frontier's changed rows.  Needs 2n bytes of
 *     scratch.
 * Other arguments, errors and support as srtc_fixpoint. */
#define SRTC_FIXPOINT_CHANGED_ROWS 1
srtc_status srtc_fixpoint_ex(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, const srtc_tensor *A,
                             srtc_tensor *X, int64_t max_iters, int32_t steps_per_check, int32_t flags,
                             int64_t *iters_out, void *stream);

/* Multi-source breadth-first levels: Section 4.2's Bellman-Ford iteration
 * X <- X (+) A (x) X taken over the boolean semiring (or, and) instead of the
 * tropical one, so level l is the step at which a vertex is first reached,
 * with a bit-packed frontier (one uint64 per vertex, bit t = source t, nsrc
 * <= 64).
 * A's pattern gives the edges (entry (i, j) = edge j -> i; values ignored).
 * sources: host array of nsrc vertex ids.  levels: device n x nsrc int32,
 * level 0 at the source, -1 if unreachable.  *depth_out (host) = largest
 * level.  Synchronizes once per level. */
srtc_status srtc_bfs_levels(srtc_ctx *ctx, const srtc_tensor *A, const int64_t *sources,
                            int32_t nsrc, int32_t *levels, int32_t *depth_out, void *stream);

/* ----------------------------------------------------------- transform -- */

/* Elementwise transforms (Section 3.4's user-defined transforms, as a fixed
 * set compiled into the library).  For every element c of C:
 *   SRTC_TF_RECIP    c = alpha / c
 *   SRTC_TF_SCALE    c = alpha * c
 *   SRTC_TF_ADD      c = c + alpha * a
 *   SRTC_TF_FMA      c = c + alpha * a * b
 *   SRTC_TF_DIV_SUM  c = c / (a + b)     (the section's nested-loop example)
 * where a = A[ia] and b = B[ib] at C's letters; A's and B's letters must be
 * letters of C (each at most once; the same extents), and a letter of C
 * missing from A or B broadcasts that operand along it, e.g.
 * D["abij"] += Ei["i"] is (SRTC_TF_ADD, alpha = 1, "i", Ei, -, -, "abij", D).
 * A and B are dense (NULL / index string ignored when the op does not use
 * them).  C is dense, or, for RECIP and SCALE only, sparse (COO or CSR: its
 * stored values are transformed, its pattern kept).  All of one value type,
 * F64 or F32; arithmetic in that type.  C is updated in place; it may not
 * overlap A or B.  Fully asynchronous. */
typedef enum srtc_transform_op {
  SRTC_TF_RECIP = 0,
  SRTC_TF_SCALE = 1,
  SRTC_TF_ADD = 2,
  SRTC_TF_FMA = 3,
  SRTC_TF_DIV_SUM = 4
} srtc_transform_op;
srtc_status srtc_transform(srtc_ctx *ctx, srtc_transform_op op, double alpha, const char *ia, const srtc_tensor *A,
                           const char *ib, const srtc_tensor *B, const char *ic, srtc_tensor *C, void *stream);

/* ------------------------------------------------------------- Jacobi -- */

/* Jacobi iteration for A x = b (Section 4.1, with the listing's slips read
 * as intended: the row sum skips the diagonal, the residual is b - A x):
 *   x^{l+1}_i = (b_i - sum_{j != i} A_ij x^l_j) / A_ii
 * from the caller's x^0 until |b - A x^l|_2 <= tol for some l >= 1 (at
 * least one update, as the listing's do-while).  A: n x n CSR (split 1) or
 * COO, F64 or F32; b, x: dense length-n vectors of the same type (device);
 * x is overwritten with that x^l.  Each step is one fused kernel (row sum,
 * update and the residual of the incoming iterate) plus a fixed-order
 * reduction; steps are replayed as captured HIP graphs of
 * `steps_per_check` steps and the host reads that many residual norms per
 * replay.  *iters_out = l, *resid_out = |b - A x^l|_2 (host, may be NULL).
 * Errors: SRTC_ERR_ARG if a row has no nonzero diagonal entry,
 * SRTC_ERR_NOT_CONVERGED if no l <= max_iters (<= 0: 10,000) qualifies (x
 * then holds x^max_iters).  Needs 3n values of scratch. */
srtc_status srtc_jacobi(srtc_ctx *ctx, const srtc_tensor *A, const srtc_tensor *b, srtc_tensor *x, double tol,
                        int64_t max_iters, int32_t steps_per_check, int64_t *iters_out, double *resid_out,
                        void *stream);

/* ---------------------------------------------------------------- apsp -- */

/* All-pairs shortest paths by Tiskin's path doubling (Section 4.2, the
 * sparsified doubling that forms P <- P (+) P_l (x) P with P_l the paths of
 * exactly l hops, l = 1, 2, 4, ... < n).  Paths are carried as SRTC_PATH64
 * values, so among equally light paths the one with fewer hops is kept.
 *   A        n x n int32 (min,+) matrix, COO or CSR; entry (i, j) is the
 *            weight of edge j -> i (repeated entries: the lightest counts).
 *            Weights must be >= 0 (SRTC_ERR_ARG otherwise); entries >= the
 *            identity are no edge.
 *   add_id   host int32 identity (NULL: INT32_MAX / 2): no path; every
 *            shortest-path weight must stay below it.
 *   D        device n x n int32, row-major: D[i, j] = weight of the lightest
 *            path j -> i (the closure of A: 0 on the diagonal), the identity
 *            where there is none.
 *   H        device n x n int32 or NULL: hops of that path, -1 where there
 *            is none (0 on the diagonal).
 *   *rounds_out (host, may be NULL) = products formed; the loop stops early
 *            once no path of exactly l hops is left.
 *   round_nnz (host, 64 slots, may be NULL): round_nnz[r] = entries of the
 *            sparse factor P_l of product r (the product forms
 *            round_nnz[r] * n path sums); unused slots are 0.
 * A's structure is always checked (SRTC_ERR_FORMAT on a malformed operand).
 * Needs 16 n^2 bytes of scratch for the two path matrices and one
 * device-to-host read per round. */
srtc_status srtc_apsp_tiskin(srtc_ctx *ctx, const void *add_id, const srtc_tensor *A, int32_t *D, int32_t *H,
                             int32_t *rounds_out, int64_t *round_nnz, void *stream);

/* -------------------------------------------------------------- batch -- */

/* Independent problems (an index shared by all three tensors, Sections
 * 3.3.1 and 5.1): C_b[ic] = A_b[ia] (x) B_b[ib] for b < ninst, in one set of
 * launches over every instance's rows (persistent work-queue kernels)
 * instead of one set per instance.
 *   ia, ib, ic  two letters per matrix, shared by all instances: A and B
 *               share one contracted letter, C = (A's other letter, B's
 *               other letter), e.g. "ik","kj","ij" or "ki","kj","ij" (A
 *               transposed).  The instance number is the implicit letter in
 *               all three tensors.
 *   As, Bs      sparse matrices (order 2, COO or CSR) of one value type;
 *               operands not already CSR in (row letter, column letter)
 *               order are folded per instance first.
 *   scheds      host int32[ninst] or NULL: instance b's SpGEMM schedule
 *               (0..SRTC_NUM_SCHEDULES-1, or -1: chosen for that instance as
 *               srtc_contract chooses).  Instances with the same schedule
 *               share each launch; the result does not depend on the
 *               schedules.  NULL: opts->schedule for all (-1: one choice for
 *               the whole batch).
 *   opts        sorted / validate / schedule as for srtc_contract (NULL:
 *               defaults).
 * Cs[b] receives CSR arrays that point into shared allocations:
 * Cs[0].rowptr/colidx/vals own the memory (free those three to release
 * every instance).  Synchronizes a few times (sizes; one features pass per
 * instance left to choose). */
srtc_status srtc_batch_contract(srtc_ctx *ctx, srtc_semiring sr, const void *add_id,
                                int32_t ninst, const srtc_tensor *As, const srtc_tensor *Bs,
                                srtc_tensor *Cs, const char *ia, const char *ib, const char *ic,
                                const srtc_schedule *scheds, const srtc_opts *opts, void *stream);

/* Exhaustive autotuner for a batch (Section 5.1's search over mappings,
 * measured, applied to the batched problem as a whole): time every schedule
 * on the batch's block-diagonal product, exactly as srtc_batch_contract
 * forms it with one schedule for every instance (median of `reps` runs
 * after one warm-up), cache the winner under that product's feature vector
 * and return it in *best, with the median times in times_ms (host
 * float[SRTC_NUM_SCHEDULES], may be NULL).  A later srtc_batch_contract of
 * the same batch with scheds = NULL and opts->schedule = -1 takes the cached
 * schedule.  Per-instance choices (srtc_autotune on each instance alone)
 * can mispredict the batch: a small instance's own time is mostly host
 * syncs and launch gaps that the batch pays once.  Arguments as
 * srtc_batch_contract (no Cs; the products are discarded).  Synchronizes
 * after every run. */
srtc_status srtc_batch_autotune(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, int32_t ninst,
                                const srtc_tensor *As, const srtc_tensor *Bs, const char *ia, const char *ib,
                                const char *ic, int32_t reps, srtc_schedule *best, float *times_ms, void *stream);

/* Batched Bellman-Ford: X_b <- X_b (+) A_b (x) X_b for every instance until
 * each is unchanged; converged instances drop out.  All X_b have the same
 * width s.  iters_out: host array of ninst step counts. */
srtc_status srtc_batch_fixpoint(srtc_ctx *ctx, srtc_semiring sr, const void *add_id,
                                int32_t ninst, const srtc_tensor *As, srtc_tensor *Xs,
                                int64_t max_iters, int32_t steps_per_check, int64_t *iters_out,
                                void *stream);

/* --------------------------------------------------------- scheduling -- */

/* The 32 scale-free features of an SpGEMM problem A (x) B (both CSR
 * matrices), the inputs of the schedule choice (Section 5.1 selects among
 * decompositions with performance models driven by sizes and nonzero
 * fractions; Section 7 proposes adjusting such models automatically).  With
 * m rows, w_i = sum over A's row i of the lengths of the B rows it meets
 * (products), out[] (host float[SRTC_NUM_FEATURES]) holds:
 *   0..9    fraction of rows of A whose length has bit length b (b >= 9 in 9)
 *   10..19  fraction of rows whose w_i has (bit length + 1) / 2 = b (bin 0:
 *           rows without products; b >= 9 in 19)
 *   20..23  log2 of m + 1, columns of B + 1, nnz(A) + 1, sum_i w_i + 1
 *   24      log2 of the compression ratio sum w / outputs over the rows
 *           floor(t m / s), t < s = min(512, m), outputs counted
 *           structurally (1 when nothing is sampled)
 *   25, 26  log2 of max_i w_i + 1 and of the longest row of A + 1
 *   27      coefficient of variation of w (population; 0 for a zero mean)
 *   28..31  one-hot of the semiring.
 * Synchronizes a few times. */
srtc_status srtc_features(srtc_ctx *ctx, srtc_semiring sr, const srtc_tensor *A,
                          const srtc_tensor *B, float *out, void *stream);

/* Exhaustive autotuner (Section 5.1's search over candidate mappings, with
 * measured instead of modelled costs): time every schedule on A (x) B
 * (median of `reps` runs after one warm-up, the paper's Section 6
 * protocol), cache the winner under the feature vector, return it in *best
 * and the median times in times_ms (host float[SRTC_NUM_SCHEDULES], may be
 * NULL). */
srtc_status srtc_autotune(srtc_ctx *ctx, srtc_semiring sr, const void *add_id,
                          const srtc_tensor *A, const srtc_tensor *B, int32_t reps,
                          srtc_schedule *best, float *times_ms, void *stream);

/* Learned selector, the automatically adjusted performance model Section 7
 * proposes (fitted to measured times instead of Section 5.1's analytic
 * models): the schedule predicted for a feature vector (host float[32]) by
 * the context's MLP (32 -> 64 -> 64 -> SRTC_NUM_SCHEDULES, ReLU), evaluated
 * on the GPU (the network stays on the device; one 128-byte upload, one
 * kernel, one 4-byte read on the context's current stream).
 * SRTC_ERR_UNSUPPORTED if no network is loaded. */
srtc_status srtc_select(srtc_ctx *ctx, const float *features, srtc_schedule *schedule);

typedef struct srtc_train_cfg {
  int32_t epochs;      /* passes over the data */
  int32_t batch;       /* minibatch size (<= 1024) */
  float lr;            /* Adam step size */
  float beta1, beta2, eps;
  uint64_t seed;       /* weight initialization and shuffling */
} srtc_train_cfg;

/* Train the selector (the performance model of srtc_select, Sections 5.1
 * and 7) on nsamples rows of features X (host, nsamples x 32) and
 * per-schedule targets T (host, nsamples x SRTC_NUM_SCHEDULES: log2 time,
 * centered per sample) with the MSE loss and Adam; forward, backward and
 * update run as HIP kernels.  Features are standardized with statistics
 * kept in the network.  A context that already holds a network continues
 * training it (weights, moments and step count).  *final_loss (host) = mean
 * loss of the last epoch.  save/load write and read the network, its
 * feature statistics and Adam state (SRTC_ERR_FORMAT: not a selector file;
 * SRTC_ERR_ARG: the file cannot be opened or written). */
srtc_status srtc_selector_train(srtc_ctx *ctx, const float *X, const float *T, int32_t nsamples,
                                const srtc_train_cfg *cfg, float *final_loss, void *stream);
srtc_status srtc_selector_save(srtc_ctx *ctx, const char *path);
srtc_status srtc_selector_load(srtc_ctx *ctx, const char *path);

/* Raw MLP kernels, for checking gradients against a reference.  All
 * pointers device, fp32, row-major.  params = [W1 (64x32), b1 (64), W2
 * (64x64), b2 (64), W3 (Kx64), b3 (K)], K = SRTC_NUM_SCHEDULES; X is
 * n x 32; Y (forward output) n x K; with T given, *loss (device) receives
 * mean over samples of sum_k (Y-T)^2 / K and grads (same layout as params)
 * its gradient. */
srtc_status srtc_mlp_forward(srtc_ctx *ctx, const float *params, const float *X, int32_t n,
                             float *Y, void *stream);
srtc_status srtc_mlp_loss_grad(srtc_ctx *ctx, const float *params, const float *X,
                               const float *T, int32_t n, float *loss, float *grads,
                               void *stream);
/* One Adam update (Kingma and Ba) of all srtc_mlp_num_params() parameters,
 * in place, as the training loop makes it:
 *   m1 = beta1 m1 + (1 - beta1) g;  m2 = beta2 m2 + (1 - beta2) g^2
 *   params -= lr (m1 / (1 - beta1^step)) / (sqrt(m2 / (1 - beta2^step)) + eps)
 * params, grads (g), m1, m2: device fp32, same layout; step >= 1 (the
 * count of updates including this one).  Fully asynchronous. */
srtc_status srtc_mlp_adam_step(srtc_ctx *ctx, float *params, const float *grads, float *m1, float *m2,
                               int64_t step, float lr, float beta1, float beta2, float eps, void *stream);
int64_t srtc_mlp_num_params(void);

#ifdef __cplusplus
}
#endif
#endif /* SRTC_H */
