// Independent problems in one set of launches.
//
// An index carried by all three tensors of a contraction enumerates
// independent problems that are best run side by side (Sections 3.3.1 and
// 5.1); running many contractions together is also the paper's closing
// suggestion (Section 7).  Here every instance's rows are laid end to end as
// one block-diagonal matrix, so each phase of the SpGEMM (symbolic, every
// numeric bin) and each fixpoint step is one persistent launch over the rows
// of all instances, pulling work from a shared atomic counter.  Instances
// that reach their fixpoint drop out of later steps.
#include <algorithm>
#include <vector>

#include "internal.hpp"
#include "spmm_plan.hpp"

using namespace srtc;

namespace {

struct InstTable {
  const int64_t *const *rowptr;
  const int32_t *const *col;
  const void *const *val;
  const int64_t *rowoff;   // ninst+1, prefix of row counts
  const int64_t *nnzoff;   // ninst+1, prefix of nnz
  const int64_t *coloff;   // column offset of each instance
  int ninst;
};

__device__ __forceinline__ int find_inst(const int64_t *off, int ninst, int64_t x) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void concat_rowptr(InstTable t, int64_t total_rows, int64_t *rp) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= total_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    if (r == total_rows) { rp[r] = t.nnzoff[t.ninst]; continue; }
    const int b = find_inst(t.rowoff, t.ninst, r);
    rp[r] = t.nnzoff[b] + t.rowptr[b][r - t.rowoff[b]];
  }
}

template <class V>
__global__ void concat_entries(InstTable t, int64_t total_nnz, int32_t *col, V *val, int32_t *row_inst) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total_nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = find_inst(t.nnzoff, t.ninst, e);
    const int64_t q = e - t.nnzoff[b];
    col[e] = (int32_t)(t.col[b][q] + t.coloff[b]);
    val[e] = reinterpret_cast<const V *>(t.val[b])[q];
  }
}

__global__ void row_instances(const int64_t *rowoff, int ninst, int64_t total_rows, int32_t *row_inst) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < total_rows;
       r += (int64_t)gridDim.x * blockDim.x)
    row_inst[r] = find_inst(rowoff, ninst, r);
}

// Per-instance CSR views of the block-diagonal result: rebased row pointers
// (instance b's m_b+1 entries start at rowoff[b] + b) and local columns.
__global__ void split_rowptr(const int64_t *rpC, const int64_t *rowoff, int ninst, int64_t total_rows,
                             int64_t *rp_out) {
  const int64_t total = total_rows + ninst;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    // g = rowoff[b] + b + i, i in [0, m_b]
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rowoff[mid] + mid <= g) lo = mid; else hi = mid - 1;
    }
    const int b = lo;
    const int64_t i = g - rowoff[b] - b;
    rp_out[g] = rpC[rowoff[b] + i] - rpC[rowoff[b]];
  }
}

__global__ void gather_instance_starts(const int64_t *rpC, const int64_t *rowoff, int ninst, int64_t *out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= ninst) out[b] = rpC[rowoff[b]];
}

template <class E>
__global__ void gather_dense(const void *const *src, const int64_t *off, int ninst, int64_t total, E *dst, int dir) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = find_inst(off, ninst, e);
    E *p = (E *)src[b];
    if (dir == 0) dst[e] = p[e - off[b]];
    else p[e - off[b]] = dst[e];
  }
}

unsigned gridn(int64_t n, int bs = 256, int64_t cap = 65536) {
  int64_t g = (n + bs - 1) / bs;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Upload a host array through pinned memory into a fresh device buffer.
template <class T> Buf upload(Ctx *c, const std::vector<T> &v, hipStream_t s) {
  Buf b(c, sizeof(T) * std::max<size_t>(v.size(), 1));
  if (!v.empty()) {
    void *pin = c->host_scratch(sizeof(T) * v.size());
    memcpy(pin, v.data(), sizeof(T) * v.size());
    SRTC_HIP(hipMemcpyAsync(b.p, pin, sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    SRTC_HIP(hipStreamSynchronize(s));
  }
  return b;
}

struct BlockDiag {
  Buf rp, col, val, row_inst, rowoff_d, coloff_d, nnzoff_d, ptrs;
  int64_t rows = 0, cols = 0, nnz = 0;
  std::vector<int64_t> rowoff, coloff, nnzoff;
  CsrView view() const {
    CsrView v;
    v.m = rows;
    v.n = cols;
    v.nnz = nnz;
    v.rowptr = rp.as<int64_t>();
    v.col = col.as<int32_t>();
    v.val = val.p;
    return v;
  }
};

void check_matrix(const srtc_tensor &t, const char *name) {
  if (t.format != SRTC_CSR || t.order != 2 || t.split != 1)
    fail(SRTC_ERR_FORMAT, std::string(name) + ": CSR matrices (order 2, split 1) required");
  if (t.nnz < 0 || !t.rowptr || (t.nnz > 0 && (!t.colidx || !t.vals))) fail(SRTC_ERR_ARG, std::string(name) + ": bad CSR");
}

CsrView view_of(const srtc_tensor &t) {
  return CsrView{t.dims[0], t.dims[1], t.nnz, t.rowptr, t.colidx, t.vals};
}

// Lay instances end to end; columns shift by col_shift[b].
void build_block_diag(Ctx *c, const std::vector<CsrView> &T, int dt, const std::vector<int64_t> &col_shift,
                      int64_t cols, BlockDiag *bd, hipStream_t s) {
  const int ninst = (int)T.size();
  bd->rowoff.assign(ninst + 1, 0);
  bd->nnzoff.assign(ninst + 1, 0);
  for (int b = 0; b < ninst; b++) {
    bd->rowoff[b + 1] = bd->rowoff[b] + T[b].m;
    bd->nnzoff[b + 1] = bd->nnzoff[b] + T[b].nnz;
  }
  bd->coloff = col_shift;
  bd->rows = bd->rowoff[ninst];
  bd->nnz = bd->nnzoff[ninst];
  bd->cols = cols;
  std::vector<uint64_t> ptrs(3 * (size_t)ninst);
  for (int b = 0; b < ninst; b++) {
    ptrs[b] = (uint64_t)T[b].rowptr;
    ptrs[ninst + b] = (uint64_t)T[b].col;
    ptrs[2 * ninst + b] = (uint64_t)T[b].val;
  }
  bd->ptrs = upload(c, ptrs, s);
  bd->rowoff_d = upload(c, bd->rowoff, s);
  bd->nnzoff_d = upload(c, bd->nnzoff, s);
  bd->coloff_d = upload(c, bd->coloff, s);
  InstTable t;
  t.rowptr = (const int64_t *const *)bd->ptrs.p;
  t.col = (const int32_t *const *)((uint64_t *)bd->ptrs.p + ninst);
  t.val = (const void *const *)((uint64_t *)bd->ptrs.p + 2 * ninst);
  t.rowoff = bd->rowoff_d.as<int64_t>();
  t.nnzoff = bd->nnzoff_d.as<int64_t>();
  t.coloff = bd->coloff_d.as<int64_t>();
  t.ninst = ninst;
  const size_t es = dtype_size(dt);
  bd->rp = Buf(c, sizeof(int64_t) * (size_t)(bd->rows + 1));
  bd->col = Buf(c, sizeof(int32_t) * (size_t)std::max<int64_t>(bd->nnz, 1));
  bd->val = Buf(c, es * (size_t)std::max<int64_t>(bd->nnz, 1));
  bd->row_inst = Buf(c, sizeof(int32_t) * (size_t)std::max<int64_t>(bd->rows, 1));
  concat_rowptr<<<gridn(bd->rows + 1), 256, 0, s>>>(t, bd->rows, bd->rp.as<int64_t>());
  SRTC_LAUNCH_CHECK("concat_rowptr");
  if (bd->nnz > 0) {
    switch (es) {
      case 8: concat_entries<uint64_t><<<gridn(bd->nnz), 256, 0, s>>>(t, bd->nnz, bd->col.as<int32_t>(), bd->val.as<uint64_t>(), nullptr); break;
      case 4: concat_entries<uint32_t><<<gridn(bd->nnz), 256, 0, s>>>(t, bd->nnz, bd->col.as<int32_t>(), bd->val.as<uint32_t>(), nullptr); break;
      default: concat_entries<uint8_t><<<gridn(bd->nnz), 256, 0, s>>>(t, bd->nnz, bd->col.as<int32_t>(), bd->val.as<uint8_t>(), nullptr); break;
    }
    SRTC_LAUNCH_CHECK("concat_entries");
  }
  if (bd->rows > 0) {
    row_instances<<<gridn(bd->rows), 256, 0, s>>>(bd->rowoff_d.as<int64_t>(), ninst, bd->rows, bd->row_inst.as<int32_t>());
    SRTC_LAUNCH_CHECK("row_instances");
  }
}

void build_block_diag(Ctx *c, const srtc_tensor *T, int ninst, const std::vector<int64_t> &col_shift, int64_t cols,
                      BlockDiag *bd, hipStream_t s) {
  std::vector<CsrView> v(ninst);
  for (int b = 0; b < ninst; b++) v[b] = view_of(T[b]);
  build_block_diag(c, v, T[0].dtype, col_shift, cols, bd, s);
}

// Row ids b0 .. b0 + n - 1 of every listed instance, laid end to end.
__global__ void fill_rows(const int64_t *__restrict__ starts, const int64_t *__restrict__ offs, int nr, int64_t total,
                          int32_t *__restrict__ rows) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = find_inst(offs, nr, e);
    rows[e] = (int32_t)(starts[r] + (e - offs[r]));
  }
}

// The operands of a batched product (srtc_batch_contract's argument rules):
// every instance as a (row letter, column letter) CSR, borrowed or folded,
// and the batch as one block-diagonal pair (A's columns follow B's row
// blocks; B keeps each instance's own columns, so C comes out with
// instance-local columns).
struct BatchOperands {
  int dt = 0;
  IdVal id{};
  std::vector<CsrOut> owned;
  std::vector<CsrView> av, bv;
  BlockDiag A, B;
};

void prepare_batch(Ctx *c, srtc_semiring sr, const void *add_id, int32_t ninst, const srtc_tensor *As,
                   const srtc_tensor *Bs, const char *ia, const char *ib, const char *ic, const srtc_schedule *scheds,
                   int validate, hipStream_t s, BatchOperands *P) {
  if (ninst <= 0 || !As || !Bs) fail(SRTC_ERR_ARG, "batch: bad arguments");
  if (!ia || !ib || !ic) fail(SRTC_ERR_INDEX, "batch: null index string");
  const std::string a(ia), b(ib), cs(ic);
  // each instance is C[ic] = A[ia] (x) B[ib] over matrices: one row, one
  // contracted and one column letter (the instance number is the letter
  // shared by all three tensors, Section 3.3.1)
  if (a.size() != 2 || b.size() != 2 || cs.size() != 2 || a[0] == a[1] || b[0] == b[1] || cs[0] == cs[1])
    fail(SRTC_ERR_INDEX, "batch: two distinct letters per matrix");
  char kk = 0;
  for (char ch : a)
    if (b.find(ch) != std::string::npos) kk = ch;
  if (!kk || cs.find(kk) != std::string::npos) fail(SRTC_ERR_INDEX, "batch: A and B must share one contracted letter");
  const char ri = a[0] == kk ? a[1] : a[0], cj = b[0] == kk ? b[1] : b[0];
  if (ri == cj || cs != std::string{ri, cj})
    fail(SRTC_ERR_INDEX, "batch: C's letters must be A's free letter, then B's");
  const int dt = As[0].dtype;
  P->dt = dt;
  P->id = make_id_public(sr, dt, add_id);
  const IdVal &id = P->id;
  for (int q = 0; q < ninst; q++) {
    for (const srtc_tensor *t : {&As[q], &Bs[q]}) {
      if (t->order != 2 || t->format == SRTC_DENSE) fail(SRTC_ERR_FORMAT, "batch: sparse matrices (COO or CSR) required");
      if (t->nnz < 0 || (t->format == SRTC_CSR && (!t->rowptr || t->split != 1)) ||
          (t->nnz > 0 && (!t->vals || (t->format == SRTC_CSR ? !t->colidx : !t->coo_keys))))
        fail(SRTC_ERR_ARG, "batch: bad sparse operand");
      if (t->dtype != dt) fail(SRTC_ERR_DTYPE, "batch: mixed value types");
      if (t->dims[0] <= 0 || t->dims[1] <= 0) fail(SRTC_ERR_DIM, "batch: nonpositive dimension");
    }
    if (As[q].dims[a[0] == kk ? 0 : 1] != Bs[q].dims[b[0] == kk ? 0 : 1])
      fail(SRTC_ERR_DIM, "batch: inner dimensions differ");
    if (scheds && (scheds[q] < -1 || scheds[q] >= SRTC_NUM_SCHEDULES)) fail(SRTC_ERR_ARG, "batch: schedule id out of range");
  }
  if (validate || c->validate_all)
    for (int q = 0; q < ninst; q++) {
      validate_operand(c, sr, &As[q], "A", s, &id);
      validate_operand(c, sr, &Bs[q], "B", s, &id);
    }
  // every operand as a (row letter, column letter) CSR: borrowed when it
  // already is one, else folded (transposed) per instance
  const std::string arow{ri}, acol{kk}, brow{kk}, bcol{cj};
  std::vector<CsrOut> &owned = P->owned;
  owned.reserve(2 * (size_t)ninst);
  std::vector<CsrView> &av = P->av, &bv = P->bv;
  av.resize(ninst);
  bv.resize(ninst);
  auto as_csr = [&](const srtc_tensor &t, const std::string &idx, const std::string &rows, const std::string &cols) {
    if (t.format == SRTC_CSR && idx == rows + cols) return view_of(t);
    std::vector<int> rm{(int)idx.find(rows[0])}, cm{(int)idx.find(cols[0])};
    const int64_t nr = t.dims[rm[0]], nc = t.dims[cm[0]];
    Buf keys(c, sizeof(int64_t) * (size_t)std::max<int64_t>(t.nnz, 1));
    const int64_t *src = t.coo_keys;
    Buf tmp;
    if (t.format == SRTC_CSR) {
      tmp = Buf(c, sizeof(int64_t) * (size_t)std::max<int64_t>(t.nnz, 1));
      csr_to_keys(view_of(t), tmp.as<int64_t>(), s);
      src = tmp.as<int64_t>();
    }
    remap_keys(c, src, t.nnz, 2, t.dims, 1, rm.data(), 1, cm.data(), keys.as<int64_t>(), s);
    owned.emplace_back();
    owned.back().kind = SCRATCH;
    fold_keys_to_csr(c, sr, dt, id, keys.as<int64_t>(), t.vals, t.nnz, nr, nc, &owned.back(), s);
    const CsrOut &f = owned.back();
    return CsrView{f.m, f.n, f.nnz, f.rowptr.as<int64_t>(), f.col.as<int32_t>(), f.val.p};
  };
  for (int q = 0; q < ninst; q++) {
    av[q] = as_csr(As[q], a, arow, acol);
    bv[q] = as_csr(Bs[q], b, brow, bcol);
  }
  // A's columns follow B's row blocks; B keeps each instance's own columns
  // (a row of A only reaches B rows of its instance), so C comes out with
  // instance-local columns and every column-width cost of the SpGEMM
  // (bitmaps, dense windows) is that of the widest instance, not of the sum
  std::vector<int64_t> a_shift(ninst), b_shift(ninst, 0);
  int64_t kt = 0, nn = 0;
  for (int q = 0; q < ninst; q++) {
    a_shift[q] = kt;
    kt += av[q].n;
    nn = std::max<int64_t>(nn, bv[q].n);
  }
  if (kt >= 0x7fffffff) fail(SRTC_ERR_UNSUPPORTED, "batch: more than 2^31-2 inner rows in total");
  build_block_diag(c, av, dt, a_shift, kt, &P->A, s);
  build_block_diag(c, bv, dt, b_shift, nn, &P->B, s);
  if (P->A.rows >= 0x7fffffff) fail(SRTC_ERR_UNSUPPORTED, "batch: more than 2^31-2 rows in total");
}

}  // namespace

extern "C" {

srtc_status srtc_batch_contract(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, int32_t ninst,
                                const srtc_tensor *As, const srtc_tensor *Bs, srtc_tensor *Cs, const char *ia,
                                const char *ib, const char *ic, const srtc_schedule *scheds, const srtc_opts *opts,
                                void *stream) {
  return guard(ctx, [&] {
    if (!Cs) fail(SRTC_ERR_ARG, "batch: bad arguments");
    srtc_opts o{-1, 1, 0, 0};
    if (opts) o = *opts;
    Ctx *c = &ctx->c;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    BatchOperands P;
    prepare_batch(c, sr, add_id, ninst, As, Bs, ia, ib, ic, scheds, o.validate, s, &P);
    const int dt = P.dt;
    const IdVal &id = P.id;
    const std::vector<CsrView> &av = P.av, &bv = P.bv;
    const BlockDiag &A = P.A, &B = P.B;
    // schedules: per instance (-1 chooses for that instance), else one for
    // the whole batch; instances sharing a schedule form one row group
    std::vector<int> isched(ninst);
    if (scheds) {
      for (int q = 0; q < ninst; q++)
        isched[q] = scheds[q] >= 0 ? scheds[q] : choose_schedule(ctx, sr, dt, av[q], bv[q], -1, s);
    } else {
      const int one = choose_schedule(ctx, sr, dt, A.view(), B.view(), o.schedule, s);
      for (int q = 0; q < ninst; q++) isched[q] = one;
    }
    CsrOut C;
    std::vector<RowGroup> groups;
    std::vector<Buf> maps;
    bool uniform = true;
    for (int q = 1; q < ninst; q++) uniform = uniform && isched[q] == isched[0];
    if (uniform) {
      spgemm(c, sr, dt, id, A.view(), B.view(), isched[0], o.sorted, &C, nullptr, s);
    } else {
      for (int k = 0; k < SRTC_NUM_SCHEDULES; k++) {
        std::vector<int64_t> starts, offs{0};
        for (int q = 0; q < ninst; q++)
          if (isched[q] == k && A.rowoff[q + 1] > A.rowoff[q]) {
            starts.push_back(A.rowoff[q]);
            offs.push_back(offs.back() + A.rowoff[q + 1] - A.rowoff[q]);
          }
        if (starts.empty()) continue;
        const int64_t nrow = offs.back();
        Buf sd = upload(c, starts, s), od = upload(c, offs, s);
        Buf rows(c, sizeof(int32_t) * (size_t)nrow);
        fill_rows<<<gridn(nrow), 256, 0, s>>>(sd.as<int64_t>(), od.as<int64_t>(), (int)starts.size(), nrow,
                                             rows.as<int32_t>());
        SRTC_LAUNCH_CHECK("fill_rows");
        groups.push_back(RowGroup{rows.as<int32_t>(), nrow, k});
        maps.push_back(std::move(rows));
      }
      spgemm_grouped(c, sr, dt, id, A.view(), B.view(), groups, o.sorted, &C, nullptr, s);
    }
    // per-instance views
    Buf rp_all(c, sizeof(int64_t) * (size_t)(A.rows + ninst), OUTPUT);
    split_rowptr<<<gridn(A.rows + ninst), 256, 0, s>>>(C.rowptr.as<int64_t>(), A.rowoff_d.as<int64_t>(), ninst, A.rows,
                                                      rp_all.as<int64_t>());
    SRTC_LAUNCH_CHECK("split_rowptr");
    Buf starts(c, sizeof(int64_t) * (size_t)(ninst + 1));
    gather_instance_starts<<<gridn(ninst + 1), 256, 0, s>>>(C.rowptr.as<int64_t>(), A.rowoff_d.as<int64_t>(), ninst,
                                                           starts.as<int64_t>());
    std::vector<int64_t> hst(ninst + 1);
    read_to_host(c, hst.data(), starts.p, sizeof(int64_t) * (size_t)(ninst + 1), s);
    const size_t es = dtype_size(dt);
    int64_t *rpa = (int64_t *)rp_all.release();
    int32_t *col = (int32_t *)C.col.release();
    char *val = (char *)C.val.release();
    for (int q = 0; q < ninst; q++) {
      srtc_tensor &out = Cs[q];
      out.order = 2;
      out.format = SRTC_CSR;
      out.dtype = dt;
      out.split = 1;
      for (int r = 0; r < SRTC_MAX_ORDER; r++) out.dims[r] = 0;
      out.dims[0] = av[q].m;
      out.dims[1] = bv[q].n;
      out.nnz = hst[q + 1] - hst[q];
      out.coo_keys = nullptr;
      out.rowptr = rpa + A.rowoff[q] + q;
      out.colidx = col + hst[q];
      out.vals = val + es * (size_t)hst[q];
    }
  });
}

srtc_status srtc_batch_autotune(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, int32_t ninst,
                                const srtc_tensor *As, const srtc_tensor *Bs, const char *ia, const char *ib,
                                const char *ic, int32_t reps, srtc_schedule *best, float *times_ms, void *stream) {
  return guard(ctx, [&] {
    Ctx *c = &ctx->c;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    BatchOperands P;
    prepare_batch(c, sr, add_id, ninst, As, Bs, ia, ib, ic, nullptr, 0, s, &P);
    // the block-diagonal pair as two CSR descriptors for the exhaustive
    // tuner, which times and caches under their features
    srtc_tensor at{}, bt{};
    const BlockDiag *blk[2] = {&P.A, &P.B};
    srtc_tensor *td[2] = {&at, &bt};
    for (int q = 0; q < 2; q++) {
      const CsrView v = blk[q]->view();
      srtc_tensor &t = *td[q];
      t.order = 2;
      t.format = SRTC_CSR;
      t.dtype = P.dt;
      t.split = 1;
      t.dims[0] = v.m;
      t.dims[1] = v.n;
      t.nnz = v.nnz;
      t.rowptr = const_cast<int64_t *>(v.rowptr);
      t.colidx = const_cast<int32_t *>(v.col);
      t.vals = const_cast<void *>(v.val);
    }
    const srtc_status st = srtc_autotune(ctx, sr, add_id, &at, &bt, reps, best, times_ms, stream);
    if (st != SRTC_OK) fail(st, c->err);
  });
}

srtc_status srtc_batch_fixpoint(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, int32_t ninst,
                                const srtc_tensor *As, srtc_tensor *Xs, int64_t max_iters, int32_t steps_per_check,
                                int64_t *iters_out, void *stream) {
  return guard(ctx, [&] {
    if (ninst <= 0 || !As || !Xs) fail(SRTC_ERR_ARG, "batch: bad arguments");
    if (sr == SRTC_PLUS_TIMES) fail(SRTC_ERR_UNSUPPORTED, "fixpoint needs an idempotent semiring");
    const int dt = As[0].dtype;
    const int64_t sw = Xs[0].order == 2 ? Xs[0].dims[1] : 1;
    int64_t nmax = 0;
    for (int b = 0; b < ninst; b++) {
      check_matrix(As[b], "A");
      if (As[b].dtype != dt || Xs[b].dtype != dt) fail(SRTC_ERR_DTYPE, "batch: mixed value types");
      if (As[b].dims[0] != As[b].dims[1]) fail(SRTC_ERR_DIM, "batch: square matrices required");
      if (Xs[b].format != SRTC_DENSE || Xs[b].dims[0] != As[b].dims[0] || (Xs[b].order == 2 ? Xs[b].dims[1] : 1) != sw)
        fail(SRTC_ERR_DIM, "batch: X_b must be dense n_b x s with one s");
      nmax = std::max<int64_t>(nmax, As[b].dims[0]);
    }
    const IdVal id = make_id_public(sr, dt, add_id);
    if (max_iters <= 0) max_iters = nmax;
    Ctx *c = &ctx->c;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    std::vector<int64_t> shift(ninst);
    int64_t nn = 0;
    for (int b = 0; b < ninst; b++) { shift[b] = nn; nn += As[b].dims[0]; }
    BlockDiag A;
    build_block_diag(c, As, ninst, shift, nn, &A, s);
    const CsrView av = A.view();
    const size_t es = dtype_size(dt);
    // dense frontiers laid end to end
    std::vector<int64_t> xoff(ninst + 1, 0);
    std::vector<uint64_t> xptr(ninst);
    for (int b = 0; b < ninst; b++) {
      xoff[b + 1] = xoff[b] + Xs[b].dims[0] * sw;
      xptr[b] = (uint64_t)Xs[b].vals;
    }
    Buf xoff_d = upload(c, xoff, s), xptr_d = upload(c, xptr, s);
    const int64_t total = xoff[ninst];
    Buf xa(c, es * (size_t)std::max<int64_t>(total, 1)), xb(c, es * (size_t)std::max<int64_t>(total, 1));
    auto move = [&](int dir) {
      if (total == 0) return;
      switch (es) {
        case 8: gather_dense<uint64_t><<<gridn(total), 256, 0, s>>>((const void *const *)xptr_d.p, xoff_d.as<int64_t>(), ninst, total, xa.as<uint64_t>(), dir); break;
        case 4: gather_dense<uint32_t><<<gridn(total), 256, 0, s>>>((const void *const *)xptr_d.p, xoff_d.as<int64_t>(), ninst, total, xa.as<uint32_t>(), dir); break;
        default: gather_dense<uint8_t><<<gridn(total), 256, 0, s>>>((const void *const *)xptr_d.p, xoff_d.as<int64_t>(), ninst, total, xa.as<uint8_t>(), dir); break;
      }
      SRTC_LAUNCH_CHECK("gather_dense");
    };
    move(0);
    SpmmPlan pl;
    pl.build(c, av, sw, s);
    int k = std::max(2, (int)steps_per_check);
    if (k % 2) k++;
    Buf flags(c, sizeof(int32_t) * (size_t)k * (size_t)(ninst + 1));
    Buf active(c, (size_t)ninst);
    std::vector<uint8_t> hact(ninst, 1);
    void *bufs[2] = {xa.p, xb.p};
    auto step = [&](int t, int parity, hipStream_t st) {
      int32_t *f = flags.as<int32_t>() + (size_t)t * (ninst + 1);
      fill_i32(f, ninst + 1, 0, st);
      spmm_with_plan(pl, sr, dt, id, av, bufs[parity], sw, bufs[parity ^ 1], 1, 0, f + ninst, A.row_inst.as<int32_t>(),
                     active.as<uint8_t>(), f, st);
    };
    hipStream_t cap;
    SRTC_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    struct Cleanup {
      hipStream_t *cap;
      hipGraph_t *g;
      hipGraphExec_t *e;
      ~Cleanup() {
        if (*e) (void)hipGraphExecDestroy(*e);
        if (*g) (void)hipGraphDestroy(*g);
        (void)hipStreamDestroy(*cap);
      }
    } cleanup{&cap, &graph, &exec};
    SRTC_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    for (int t = 0; t < k; t++) step(t, t & 1, cap);
    SRTC_HIP(hipStreamEndCapture(cap, &graph));
    SRTC_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    std::vector<int64_t> iters(ninst, 0);
    std::vector<int32_t> hf((size_t)k * (ninst + 1));
    int remaining = ninst;
    int64_t r = 0;
    while (r < max_iters && remaining > 0) {
      void *pin = c->host_scratch((size_t)ninst);
      memcpy(pin, hact.data(), (size_t)ninst);
      SRTC_HIP(hipMemcpyAsync(active.p, pin, (size_t)ninst, hipMemcpyHostToDevice, s));
      int nsteps;
      if (r + k <= max_iters) {
        SRTC_HIP(hipGraphLaunch(exec, s));
        nsteps = k;
      } else {
        nsteps = (int)(max_iters - r);
        for (int t = 0; t < nsteps; t++) step(t, t & 1, s);
        if (nsteps & 1) SRTC_HIP(hipMemcpyAsync(xa.p, xb.p, es * (size_t)total, hipMemcpyDeviceToDevice, s));
      }
      read_to_host(c, hf.data(), flags.p, sizeof(int32_t) * (size_t)nsteps * (ninst + 1), s);
      for (int b = 0; b < ninst; b++) {
        if (!hact[b]) continue;
        for (int t = 0; t < nsteps; t++) {
          if (hf[(size_t)t * (ninst + 1) + b] == 0) {
            iters[b] = r + t + 1;
            hact[b] = 0;
            remaining--;
            break;
          }
        }
      }
      r += nsteps;
    }
    move(1);
    bool all = true;
    for (int b = 0; b < ninst; b++) {
      if (hact[b]) { iters[b] = r; all = false; }
      if (iters_out) iters_out[b] = iters[b];
    }
    SRTC_HIP(hipStreamSynchronize(s));
    if (!all) fail(SRTC_ERR_NOT_CONVERGED, "some instance still changing after max_iters steps");
  });
}

}  // extern "C"
