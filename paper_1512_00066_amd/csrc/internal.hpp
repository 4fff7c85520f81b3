// Host-side internal interfaces between the C-ABI layer and the kernels.
#pragma once

#include <map>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace srtc {

struct Mlp;  // selector network (mlp.hip)

struct Ctx {
  int device = 0;
  srtc_alloc_fn alloc = nullptr;
  srtc_free_fn free_fn = nullptr;
  void *user = nullptr;
  std::string err = "no error";
  int num_cus = 256;
  size_t lds_per_block = 65536;
  // autotune cache: feature fingerprint -> schedule
  std::map<std::string, int> tune_cache;
  Mlp *mlp = nullptr;
  // pinned host scratch for small device->host reads
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
  // stream of the call in progress (kernels and scratch reuse follow it)
  hipStream_t stream = nullptr;
  // scratch cache used when no allocator callback is given: freed scratch
  // blocks are kept by power-of-two size class and reused in stream order
  std::map<void *, int> block_class;
  std::vector<std::vector<void *>> free_blocks = std::vector<std::vector<void *>>(64);
  hipStream_t cache_stream = nullptr;
  bool trace = false;
  // environment switches read at context creation: SRTC_VALIDATE (check
  // every sparse operand's structure), SRTC_FORCE_SCHEDULE (the SpGEMM
  // schedule of every product whose caller leaves the choice open) and
  // SRTC_LDS_BUDGET (bytes of LDS a SpGEMM kernel may use per block)
  bool validate_all = false;
  int force_schedule = -1;
  int64_t lds_budget = 160 * 1024;
  // column blocks of B for wide products (SRTC_COL_BLOCKS): -1 or 1 = none,
  // 0 = sized from B, q >= 2 = q blocks
  int col_blocks = -1;
  // hub tile size of sparse x sparse (+,x) products (SRTC_HUB_TILE): 0 = none
  int hub_tile = 0;
  // this device's fixed buffer of srtc_contract_noalloc (device address)
  void *fixed_scratch = nullptr;
  // Tables built from B alone (window tables, value records), kept while one
  // B multiplies several A's (the row panels of srtc_contract_panels, whose
  // folded B stays allocated and unchanged throughout): keep_b names that B
  // (rowptr null: nothing is kept), b_tables holds what was built from it,
  // by key (a window width; -1 for the value records).
  struct KeptB {
    const int64_t *rowptr = nullptr;
    const int32_t *col = nullptr;
    const void *val = nullptr;
    int64_t m = 0, n = 0, nnz = 0;
  };
  struct BTable {
    int64_t key;
    Buf buf;
  };
  KeptB keep_b;
  std::vector<BTable> b_tables;
  void release_cache();
  void tracef(const char *fmt, ...);
  // per-kernel profile: HIP events around each launch on its stream, with
  // the launch's algorithmic bytes; resolved when queried
  struct ProfPending {
    int slot;
    hipEvent_t e0, e1;
    double bytes;
  };
  struct ProfAgg {
    std::string name;
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
  };
  bool profiling = false;
  std::vector<ProfPending> prof_pending;
  std::vector<ProfAgg> prof;
  std::vector<hipEvent_t> event_pool;
  void prof_resolve();

  void *raw_alloc(size_t bytes, int kind);
  void raw_free(void *p, int kind);
  void *host_scratch(size_t bytes);
};

// Records the enclosed launches as one profiled kernel (no-op unless
// profiling is on, or while the stream is being captured into a graph).
struct ProfScope {
  Ctx *c = nullptr;
  int slot = -1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double bytes = 0;
  hipStream_t s = nullptr;
  ProfScope(Ctx *ctx, const char *name, double algorithmic_bytes, hipStream_t stream);
  ~ProfScope();
};

// A device CSR matrix view (not owning).
struct CsrView {
  int64_t m = 0, n = 0, nnz = 0;
  const int64_t *rowptr = nullptr;
  const int32_t *col = nullptr;
  const void *val = nullptr;
};

// An owned CSR result (kind: OUTPUT for results handed to the caller,
// SCRATCH for intermediates such as folded operands).
struct CsrOut {
  int64_t m = 0, n = 0, nnz = 0;
  int kind = OUTPUT;
  Buf rowptr, col, val;
};

// ---------------------------------------------------------------- prims --
// out[i] = sum_{j<i} in[i]; out has n+1 entries (out[n] = total).  In = int32
// or int64.  Returns nothing; total stays on device.
void excl_scan_i64(Ctx *c, const int64_t *in, int64_t *out, int64_t n, hipStream_t s);
void excl_scan_i32(Ctx *c, const int32_t *in, int64_t *out, int64_t n, hipStream_t s);
// The same scan with its tile sums in caller memory (excl_scan_workspace(n)
// int64 values); allocates nothing.
int64_t excl_scan_workspace(int64_t n);
void excl_scan_i64_ws(const int64_t *in, int64_t *out, int64_t n, int64_t *sums, hipStream_t s);
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);
void fill_bytes_value(void *p, int64_t n, int dtype, IdVal v, hipStream_t s);
int64_t read_i64(Ctx *c, const int64_t *dev, hipStream_t s);
void read_to_host(Ctx *c, void *host, const void *dev, size_t bytes, hipStream_t s);

// ----------------------------------------------------------------- fold --
// Keys (row*ncols + col, < 2^63) with values -> CSR, duplicates combined in
// input order, identity entries dropped.  Synchronizes once.
void fold_keys_to_csr(Ctx *c, int sr, int dt, IdVal id, const int64_t *keys, const void *vals,
                      int64_t nnz, int64_t nrows, int64_t ncols, CsrOut *out, hipStream_t s);
// Mode remap of linearized keys: out[t] = rowkey*ncols + colkey where the
// row (col) key linearizes the listed source modes.
void remap_keys(Ctx *c, const int64_t *keys, int64_t nnz, int order, const int64_t *dims,
                int nrow_modes, const int *row_modes, int ncol_modes, const int *col_modes,
                int64_t *out, hipStream_t s);
// Expand a CSR matrix to linearized keys row*ncols+col.
void csr_to_keys(const CsrView &a, int64_t *keys, hipStream_t s);
// Stable LSD radix sort of 64-bit keys carrying a 32-bit payload (exposed
// for tests through the fold).
void radix_sort_pairs(Ctx *c, int64_t *keys, uint32_t *payload, int64_t n, int bits,
                      hipStream_t s);

// --------------------------------------------------------------- spgemm --
struct Schedule {
  // symbolic: rows with products <= sym_hash_max use an LDS hash, others a
  // bitmap
  int64_t sym_hash_max;
  // numeric bins by exact row nnz: <= t_tiny (64-slot hash), <= t_small
  // (512-slot hash), <= t_mid (4096-slot hash), <= t_big (8192-slot hash),
  // above: dense LDS windows
  int64_t t_tiny, t_small, t_mid, t_big;
  int small_wave;    // 512-slot bin: one 64-thread wave per row (1) or two waves (0)
  int dense_bs;      // dense-window block size (256 or 512; the widest windows always take 1024)
  int dense_wide;    // dense window of 8K (0), 16K (1) or 4K (2) 8-byte accumulators
};
const Schedule &schedule(int id);

struct SpgemmStats {
  int64_t products = 0;
  int64_t nnz = 0;
  int64_t dense_rows = 0;
  int compacted = 0;
};

// C = A (x) B, output CSR with ascending columns (sorted=1) allocated from
// the context.  Synchronizes a few times (bin sizes, output size, flags).
void spgemm(Ctx *c, int sr, int dt, IdVal id, const CsrView &A, const CsrView &B, int sched,
            int sorted, CsrOut *out, SpgemmStats *st, hipStream_t s);
// Rows of A multiplied under their own schedules: group g covers the rows
// listed in row_map (device, nsel ids; every row of A belongs to at most one
// group, rows in none get no entries).  One output, as spgemm().
struct RowGroup {
  const int32_t *row_map;
  int64_t nsel;
  int sched;
};
void spgemm_grouped(Ctx *c, int sr, int dt, IdVal id, const CsrView &A, const CsrView &B,
                    const std::vector<RowGroup> &groups, int sorted, CsrOut *out, SpgemmStats *st,
                    hipStream_t s);
// C = M (.) (A (x) B) over M's pattern (sorted rows; identity results dropped).
void spgemm_masked(Ctx *c, int sr, int dt, IdVal id, const CsrView &A, const CsrView &B, const CsrView &M,
                   CsrOut *out, hipStream_t s);
// C = A (x) B over (+,x) with the block of the `hub` densest rows of A,
// inner indices and columns of B formed on the matrix cores and the rest
// sparsely (one augmented product); the same output as spgemm().
bool hub_product_applies(int sr, int dt, const CsrView &A, const CsrView &B, int64_t hub);
void spgemm_hubs(Ctx *c, int dt, IdVal id, const CsrView &A, const CsrView &B, int64_t hub, int sched,
                 int sorted, CsrOut *out, SpgemmStats *st, hipStream_t s);
// Row product counts w_i (int64, m entries).
void row_products(const CsrView &A, const CsrView &B, int64_t *w, hipStream_t s);
// C = X (+) Y for two CSR matrices of the same shape (sorted rows); the
// union of patterns, identity results dropped.  Synchronizes once.
void ewise_add(Ctx *c, int sr, int dt, IdVal id, const CsrView &X, const CsrView &Y, CsrOut *out,
               hipStream_t s);

// ----------------------------------------------------------------- spmm --
// Y[i,:] = [X0[i,:] (+)] (+)_k A_ik (x) X[k,:]; dense row-major width s.
// accumulate: Y's previous contents join the sum.  changed (optional, device
// int) is set to 1 if any Y entry differs from X0 (self-term form).
void spmm(Ctx *c, int sr, int dt, IdVal id, const CsrView &A, const void *X, int64_t s_width,
          void *Y, int accumulate, hipStream_t s);
void bf_step(int sr, int dt, IdVal id, const CsrView &A, const void *X, void *Y, int64_t s_width,
             int32_t *changed, const int32_t *row_inst, const uint8_t *inst_active,
             int32_t *inst_changed, hipStream_t s);
void bfs_step(const CsrView &A, const uint64_t *front, uint64_t *visited, uint64_t *next,
              int32_t *levels, int nsrc, int level, int32_t *changed, hipStream_t s);

// ----------------------------------------------------------------- apsp --
// Tiskin's path doubling over packed (weight, hops) paths: D = closure of A
// (dense n x n int32, idw where unreachable), H = hops of the kept path
// (optional, -1 where unreachable), *rounds = products formed, round_nnz
// (host, 64 slots, optional) = entries of each round's sparse factor.
void apsp_tiskin(Ctx *c, const CsrView &A, int32_t idw, int32_t *D, int32_t *H, int32_t *rounds, int64_t *round_nnz,
                 hipStream_t s);

// --------------------------------------------------------------- dense --
// C_z = A_z B_z (+ C_z with accumulate) for z < batch, each row-major and
// the batches contiguous (strides MK, KN, MN).
void dense_gemm_plus_times(Ctx *c, int dt, const void *A, const void *B, void *C, int64_t M,
                           int64_t N, int64_t K, int accumulate, hipStream_t s, int64_t batch = 1);
// dst mode q = src mode perm[q] (dims: src extents, last mode fastest).
void dense_permute(const void *src, void *dst, int esize, int order, const int64_t *dims,
                   const int *perm, hipStream_t s);
// C = A (x) B elementwise over n entries ((+) with C's old values when
// accumulating).
void dense_hadamard(int sr, int dt, IdVal id, const void *A, const void *B, void *C, int64_t n, int accumulate,
                    hipStream_t s);
// The same with dst's previous values joining by the semiring's (+).
void dense_permute_combine(int sr, int dt, IdVal id, const void *src, void *dst, int order,
                           const int64_t *dims, const int *perm, hipStream_t s);

// ------------------------------------------------------------ transform --
// C (dense, order `order`, extents cext) updated elementwise by transform
// `op` (srtc_transform_op) with A and B read at stride sa[q] / sb[q] along
// C's mode q (0 broadcasts; A or B may be null when the op ignores it).
void transform_dense_call(int op, int dt, double alpha, const int64_t *cext, int order, const void *A,
                          const int64_t *sa, const void *B, const int64_t *sb, void *C, hipStream_t s);

// Jacobi iteration on an n x n CSR A: the inverse-free diagonal d, the
// lanes per row and the fixed grid whose per-block residual partials are
// summed in a fixed order.
struct JacobiPlan {
  Ctx *ctx = nullptr;
  int dt = SRTC_F64;
  CsrView A;
  int G = 32;
  int grid = 1;
  Buf dbuf, part;
  // fails with SRTC_ERR_ARG when a row has no nonzero diagonal entry
  void build(Ctx *c, int dt, const CsrView &A, hipStream_t s);
};
// Device state of a Jacobi solve: iter = l of the current iterate x^l,
// done = 1 once |b - A x^l|^2 <= tol^2 with l >= 1 (rsq = that value; while
// running, the last residual formed).
struct JacobiState {
  int64_t iter;
  int32_t done;
  int32_t pad;
  double rsq;
};
// Unless st->done: x_out = (b - (A - diag) x_in) / diag, then the residual
// of x_in decides whether to stop (x_in kept) or advance st->iter.
void jacobi_step_call(const JacobiPlan &pl, const void *b, const void *x_in, void *x_out, JacobiState *st,
                      double tol2, hipStream_t s);

// ------------------------------------------------------------- features --
void spgemm_features(Ctx *c, int sr, int dt, const CsrView &A, const CsrView &B, float *out,
                     hipStream_t s);

// The schedule of an SpGEMM A (x) B: `requested` if >= 0, else the
// environment's forced one, else the autotune cache, the learned selector
// or schedule 0 (features are computed only when a cache or network exists).
int choose_schedule(srtc_ctx *ctx, int sr, int dt, const CsrView &A, const CsrView &B, int requested, hipStream_t s);

// The caller's additive identity checked against the semiring, or the
// default identity (Section 3.1).
IdVal make_id_public(int sr, int dt, const void *add_id);
// Key of the autotune cache for a feature vector.
std::string tune_key(int sr, int dt, const float *features);
// Structure checks of a sparse operand (SRTC_ERR_FORMAT on failure); one
// host sync.
void validate_operand(Ctx *c, int sr, const srtc_tensor *t, const char *name, hipStream_t s,
                      const IdVal *id = nullptr);

}  // namespace srtc

struct srtc_ctx {
  srtc::Ctx c;
};

namespace srtc {
// The context's stream is saved and restored, so an entry point called from
// inside another keeps the outer call's stream for its scratch memory.
template <class F> srtc_status guard(srtc_ctx *ctx, F &&f) {
  if (!ctx) return SRTC_ERR_ARG;
  struct Restore {
    Ctx *c;
    hipStream_t s;
    ~Restore() { c->stream = s; }
  } restore{&ctx->c, ctx->c.stream};
  try {
    SRTC_HIP(hipSetDevice(ctx->c.device));
    f();
    return SRTC_OK;
  } catch (const Error &e) {
    ctx->c.err = e.msg;
    return e.st;
  } catch (const std::bad_alloc &) {
    ctx->c.err = "host allocation failed";
    return SRTC_ERR_OOM;
  } catch (...) {
    ctx->c.err = "internal error";
    return SRTC_ERR_DEVICE;
  }
}
}  // namespace srtc
