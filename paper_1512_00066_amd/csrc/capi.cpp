// C-ABI entry points of libsrtc (declared in include/srtc.h).
//
// This layer validates arguments, turns index strings into a fold plan
// (Section 5.1: each index of a contraction is a batch, row, inner or column
// index according to which tensors carry it, Section 3.3.1), and dispatches
// to the kernels.  No exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "spmm_plan.hpp"

namespace srtc {

// ------------------------------------------------------------- memory --
// Device memory.  With an allocator callback every buffer (output or
// scratch) comes from it -- a caching, stream-ordered allocator such as
// torch's is expected.  Without one, outputs come from hipMalloc and scratch
// from a per-context cache of hipMalloc blocks (power-of-two size classes),
// reused in the order of the context's stream; a call on a different stream
// first waits for the previous one.
static int size_class(size_t bytes) {
  int c = 8;  // 256 bytes minimum
  while (((size_t)1 << c) < bytes) c++;
  return c;
}

void Ctx::release_cache() {
  if (block_class.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto &kv : block_class) (void)hipFree(kv.first);
  block_class.clear();
  for (auto &v : free_blocks) v.clear();
}

void *Ctx::raw_alloc(size_t bytes, int kind) {
  if (bytes == 0) bytes = 1;
  void *p = nullptr;
  if (alloc) {
    p = alloc(user, bytes);
  } else if (kind == OUTPUT) {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      release_cache();
      if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    }
  } else {
    if (cache_stream != stream) {
      // blocks freed on the previous stream may still be in use there
      SRTC_HIP(hipStreamSynchronize(cache_stream));
      cache_stream = stream;
    }
    const int c = size_class(bytes);
    if (!free_blocks[c].empty()) {
      p = free_blocks[c].back();
      free_blocks[c].pop_back();
    } else {
      if (hipMalloc(&p, (size_t)1 << c) != hipSuccess) {
        release_cache();
        if (hipMalloc(&p, (size_t)1 << c) != hipSuccess) p = nullptr;
      }
      if (p) block_class[p] = c;
    }
  }
  if (!p) fail(SRTC_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  return p;
}

void Ctx::raw_free(void *p, int kind) {
  if (!p) return;
  if (free_fn) {
    free_fn(user, p);
  } else if (kind == OUTPUT) {
    (void)hipFree(p);
  } else {
    auto it = block_class.find(p);
    if (it != block_class.end()) free_blocks[it->second].push_back(p);
  }
}

void Ctx::tracef(const char *fmt, ...) {
  if (!trace) return;
  va_list ap;
  va_start(ap, fmt);
  fprintf(stderr, "[srtc] ");
  vfprintf(stderr, fmt, ap);
  fprintf(stderr, "\n");
  fflush(stderr);
  va_end(ap);
}

void *Ctx::host_scratch(size_t bytes) {
  if (bytes > pinned_bytes) {
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    size_t nb = std::max<size_t>(bytes, 1 << 16);
    SRTC_HIP(hipHostMalloc(&pinned, nb, hipHostMallocDefault));
    pinned_bytes = nb;
  }
  return pinned;
}

// ------------------------------------------------------------ profile --
static hipEvent_t take_event(Ctx *c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  SRTC_HIP(hipEventCreate(&e));
  return e;
}

ProfScope::ProfScope(Ctx *ctx, const char *name, double algorithmic_bytes, hipStream_t stream)
    : c(ctx), bytes(algorithmic_bytes), s(stream) {
  if (!c || !c->profiling) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  for (size_t q = 0; q < c->prof.size(); q++)
    if (c->prof[q].name == name) slot = (int)q;
  if (slot < 0) {
    c->prof.push_back(Ctx::ProfAgg{name});
    slot = (int)c->prof.size() - 1;
  }
  e0 = take_event(c);
  e1 = take_event(c);
  SRTC_HIP(hipEventRecord(e0, s));
}

ProfScope::~ProfScope() {
  if (slot < 0) return;
  if (hipEventRecord(e1, s) == hipSuccess) c->prof_pending.push_back(Ctx::ProfPending{slot, e0, e1, bytes});
  if (c->prof_pending.size() > 4096) {
    try { c->prof_resolve(); } catch (...) {}
  }
}

void Ctx::prof_resolve() {
  for (auto &p : prof_pending) {
    SRTC_HIP(hipEventSynchronize(p.e1));
    float ms = 0.f;
    SRTC_HIP(hipEventElapsedTime(&ms, p.e0, p.e1));
    prof[p.slot].launches++;
    prof[p.slot].ms += ms;
    prof[p.slot].bytes += p.bytes;
    event_pool.push_back(p.e0);
    event_pool.push_back(p.e1);
  }
  prof_pending.clear();
}

Buf::Buf(Ctx *c, size_t n, int k) : ctx(c), p(nullptr), bytes(n), kind(k) { p = c->raw_alloc(n, k); }
Buf &Buf::operator=(Buf &&o) noexcept {
  if (this != &o) {
    if (p && ctx) ctx->raw_free(p, kind);
    ctx = o.ctx;
    p = o.p;
    bytes = o.bytes;
    kind = o.kind;
    o.p = nullptr;
  }
  return *this;
}
Buf::~Buf() {
  if (p && ctx) ctx->raw_free(p, kind);
}

void mlp_destroy(Mlp *m);  // mlp.hip

namespace {

// ------------------------------------------------------------ helpers --
bool semiring_ok(int sr, int dt) {
  switch (sr) {
    case SRTC_PLUS_TIMES: return dt == SRTC_F64 || dt == SRTC_F32;
    case SRTC_MIN_PLUS: return dt == SRTC_I32 || dt == SRTC_F32 || dt == SRTC_PATH64;
    case SRTC_OR_AND: return dt == SRTC_BOOL8;
    case SRTC_MAX_TIMES: return dt == SRTC_F32 || dt == SRTC_F64;
  }
  return false;
}

// The additive identity: the caller's value or the default (Section 3.1).
IdVal make_id(int sr, int dt, const void *add_id) {
  if (sr < 0 || sr > 3) fail(SRTC_ERR_ARG, "unknown semiring");
  if (!semiring_ok(sr, dt)) fail(SRTC_ERR_DTYPE, "value type not defined for this semiring");
  IdVal v{0.0, 0};
  switch (sr) {
    case SRTC_PLUS_TIMES: {
      double x = 0.0;
      if (add_id) x = dt == SRTC_F64 ? *(const double *)add_id : (double)*(const float *)add_id;
      if (x != 0.0) fail(SRTC_ERR_ARG, "(+,x) additive identity must be 0");
      break;
    }
    case SRTC_MIN_PLUS:
      if (dt == SRTC_I32) {
        v.i = add_id ? *(const int32_t *)add_id : (int32_t)(INT32_MAX / 2);
        // a product of two operands in [-id, id] then stays inside int32
        if (v.i <= 0 || v.i > INT32_MAX / 2)
          fail(SRTC_ERR_ARG, "(min,+) int identity must lie in 1..INT32_MAX/2");
      } else if (dt == SRTC_PATH64) {
        // a packed path: the identity's weight (its hop count must be 0)
        const uint64_t pv = add_id ? *(const uint64_t *)add_id : (uint64_t)(INT32_MAX / 2) << 32;
        if ((pv & 0xffffffffull) != 0 || (pv >> 32) == 0 || (pv >> 32) > (uint64_t)(INT32_MAX / 2))
          fail(SRTC_ERR_ARG, "(min,+) path identity must be (weight in 1..INT32_MAX/2, 0 hops)");
        v.i = (int64_t)(pv >> 32);
      } else {
        v.f = add_id ? (double)*(const float *)add_id : (double)std::numeric_limits<float>::infinity();
      }
      break;
    case SRTC_OR_AND:
      if (add_id && *(const uint8_t *)add_id != 0) fail(SRTC_ERR_ARG, "(or,and) identity must be false");
      break;
    case SRTC_MAX_TIMES:
      if (add_id) v.f = dt == SRTC_F64 ? *(const double *)add_id : (double)*(const float *)add_id;
      break;
  }
  return v;
}

int64_t prod_dims(const srtc_tensor *t) {
  int64_t p = 1;
  for (int i = 0; i < t->order; i++) p *= t->dims[i];
  return p;
}

void check_tensor(const srtc_tensor *t, const char *name) {
  if (!t) fail(SRTC_ERR_ARG, std::string(name) + ": null tensor");
  if (t->order < 0 || t->order > SRTC_MAX_ORDER) fail(SRTC_ERR_ARG, std::string(name) + ": bad order");
  for (int i = 0; i < t->order; i++)
    if (t->dims[i] <= 0) fail(SRTC_ERR_DIM, std::string(name) + ": nonpositive dimension");
  if (t->format < SRTC_DENSE || t->format > SRTC_CSR) fail(SRTC_ERR_ARG, std::string(name) + ": bad format");
  if (t->format != SRTC_DENSE && t->nnz < 0) fail(SRTC_ERR_ARG, std::string(name) + ": negative nnz");
  if (t->format == SRTC_COO && t->nnz > 0 && (!t->coo_keys || !t->vals))
    fail(SRTC_ERR_ARG, std::string(name) + ": COO without keys/values");
  if (t->format == SRTC_CSR) {
    if (!t->rowptr) fail(SRTC_ERR_ARG, std::string(name) + ": CSR without rowptr");
    if (t->nnz > 0 && (!t->colidx || !t->vals)) fail(SRTC_ERR_ARG, std::string(name) + ": CSR without cols/values");
    if (t->split < 0 || t->split > t->order) fail(SRTC_ERR_ARG, std::string(name) + ": bad split");
  }
  if (t->format == SRTC_DENSE && prod_dims(t) > 0 && !t->vals) fail(SRTC_ERR_ARG, std::string(name) + ": no values");
}

std::string letters(const char *s, const srtc_tensor *t, const char *name) {
  if (!s) fail(SRTC_ERR_INDEX, std::string(name) + ": null index string");
  std::string r(s);
  if ((int)r.size() != t->order) fail(SRTC_ERR_INDEX, std::string(name) + ": index string length differs from order");
  for (size_t i = 0; i < r.size(); i++)
    for (size_t j = i + 1; j < r.size(); j++)
      if (r[i] == r[j]) fail(SRTC_ERR_INDEX, std::string(name) + ": repeated index (diagonals are not supported)");
  return r;
}

int64_t row_extent(const srtc_tensor *t) {
  int64_t r = 1;
  for (int i = 0; i < t->split; i++) r *= t->dims[i];
  return r;
}

CsrView csr_view(const srtc_tensor *t) {
  CsrView v;
  v.m = row_extent(t);
  v.n = 1;
  for (int i = t->split; i < t->order; i++) v.n *= t->dims[i];
  v.nnz = t->nnz;
  v.rowptr = t->rowptr;
  v.col = t->colidx;
  v.val = t->vals;
  return v;
}

// Fold a sparse tensor (COO or CSR) to a CSR matrix with the given row and
// column letters; returns a view (borrowed if the layout already matches).
struct Folded {
  CsrOut own;
  CsrView view;
  bool owned = false;
};

void fold_sparse(Ctx *c, int sr, IdVal id, const srtc_tensor *t, const std::string &idx, const std::string &rows,
                 const std::string &cols, Folded *f, hipStream_t s, bool force = false) {
  if (!force && t->format == SRTC_CSR && idx == rows + cols && t->split == (int)rows.size()) {
    f->view = csr_view(t);
    f->owned = false;
    return;
  }
  std::vector<int> rm, cm;
  for (char ch : rows) rm.push_back((int)idx.find(ch));
  for (char ch : cols) cm.push_back((int)idx.find(ch));
  int64_t nr = 1, nc = 1;
  for (int q : rm) nr *= t->dims[q];
  for (int q : cm) nc *= t->dims[q];
  const int64_t nnz = t->nnz;
  Buf keys(c, sizeof(int64_t) * (size_t)std::max<int64_t>(nnz, 1));
  const int64_t *src_keys = t->coo_keys;
  Buf tmp;
  if (t->format == SRTC_CSR) {
    CsrView v = csr_view(t);
    tmp = Buf(c, sizeof(int64_t) * (size_t)std::max<int64_t>(nnz, 1));
    csr_to_keys(v, tmp.as<int64_t>(), s);
    src_keys = tmp.as<int64_t>();
  }
  remap_keys(c, src_keys, nnz, t->order, t->dims, (int)rm.size(), rm.data(), (int)cm.size(), cm.data(),
             keys.as<int64_t>(), s);
  if (!force) f->own.kind = SCRATCH;
  fold_keys_to_csr(c, sr, t->dtype, id, keys.as<int64_t>(), t->vals, nnz, nr, nc, &f->own, s);
  f->owned = true;
  f->view.m = f->own.m;
  f->view.n = f->own.n;
  f->view.nnz = f->own.nnz;
  f->view.rowptr = f->own.rowptr.as<int64_t>();
  f->view.col = f->own.col.as<int32_t>();
  f->view.val = f->own.val.p;
}

void set_csr_out(srtc_tensor *out, CsrOut &o, int order, const int64_t *dims, int split, int dtype) {
  out->order = order;
  for (int i = 0; i < SRTC_MAX_ORDER; i++) out->dims[i] = i < order ? dims[i] : 0;
  out->format = SRTC_CSR;
  out->dtype = dtype;
  out->split = split;
  out->nnz = o.nnz;
  out->coo_keys = nullptr;
  out->rowptr = (int64_t *)o.rowptr.release();
  out->colidx = (int32_t *)o.col.release();
  out->vals = o.val.release();
}

bool overlaps(const void *a, size_t an, const void *b, size_t bn) {
  if (!a || !b || an == 0 || bn == 0) return false;
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + bn && y < x + an;
}

size_t tensor_value_bytes(const srtc_tensor *t) {
  const size_t es = dtype_size(t->dtype);
  if (t->format == SRTC_DENSE) return es * (size_t)prod_dims(t);
  return es * (size_t)t->nnz;
}

__global__ void col_mod_kernel(int32_t *col, int64_t n, int64_t mod) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    col[i] = (int32_t)(col[i] % mod);
}

// ------------------------------------------------------------- planning --
struct Plan {
  std::string batch, M, K, N;  // letters
  std::map<char, int64_t> dim;
};

Plan plan_contraction(const std::string &a, const srtc_tensor *A, const std::string &b, const srtc_tensor *B,
                      const std::string &cidx, const srtc_tensor *C) {
  Plan p;
  auto add_dims = [&](const std::string &s, const srtc_tensor *t) {
    for (size_t i = 0; i < s.size(); i++) {
      auto it = p.dim.find(s[i]);
      if (it == p.dim.end()) p.dim[s[i]] = t->dims[i];
      else if (it->second != t->dims[i]) fail(SRTC_ERR_DIM, std::string("index '") + s[i] + "' has two extents");
    }
  };
  add_dims(a, A);
  add_dims(b, B);
  add_dims(cidx, C);
  for (char ch : cidx) {
    const bool ia = a.find(ch) != std::string::npos, ib = b.find(ch) != std::string::npos;
    if (ia && ib) p.batch += ch;
    else if (ia) p.M += ch;
    else if (ib) p.N += ch;
    else fail(SRTC_ERR_INDEX, std::string("index '") + ch + "' appears only in the output");
  }
  for (char ch : a) {
    const bool ib = b.find(ch) != std::string::npos, ic = cidx.find(ch) != std::string::npos;
    if (ib && !ic) p.K += ch;
    else if (!ib && !ic) fail(SRTC_ERR_INDEX, std::string("index '") + ch + "' appears only in A (reduction)");
  }
  for (char ch : b)
    if (a.find(ch) == std::string::npos && cidx.find(ch) == std::string::npos)
      fail(SRTC_ERR_INDEX, std::string("index '") + ch + "' appears only in B (reduction)");
  return p;
}

int64_t extent(const Plan &p, const std::string &s) {
  int64_t e = 1;
  for (char ch : s) e *= p.dim.at(ch);
  return e;
}

std::string rows_of_c(const std::string &cidx, const Plan &p) {
  std::string r;
  for (char ch : cidx)
    if (p.N.find(ch) == std::string::npos) r += ch;
  return r;
}

__global__ void bfs_init(const int64_t *src, int nsrc, uint64_t *front, uint64_t *visited, int32_t *levels) {
  const int t = threadIdx.x;
  if (t < nsrc) {
    atomicOr((unsigned long long *)&front[src[t]], 1ull << t);
    atomicOr((unsigned long long *)&visited[src[t]], 1ull << t);
    levels[src[t] * nsrc + t] = 0;
  }
}

// ---------------------------------------------------- accumulate (+=) --
// C_new = C_old (+) A (x) B as one product: A' = [A | I] and B' = [B ; C_old]
// give A' (x) B' = A (x) B (+) I (x) C_old, and I (x) C_old = C_old because
// the identity's entries are the multiplicative identity.  Each row's
// accumulator thus starts from (holds) the old row's values, the symbolic
// pass counts the union of patterns, and no sort is needed.
__global__ void aug_a_rowptr(const int64_t *__restrict__ rpA, int64_t m, int64_t *__restrict__ rp) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= m; i += (int64_t)gridDim.x * blockDim.x)
    rp[i] = rpA[i] - rpA[0] + i;
}

template <class V>
__global__ void aug_a_entries(const int64_t *__restrict__ rpA, const int32_t *__restrict__ cA, const V *__restrict__ vA,
                              int64_t m, int64_t k, V one, const int64_t *__restrict__ rp, int32_t *__restrict__ col,
                              V *__restrict__ val) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t i = wid; i < m; i += nw) {
    const int64_t a = rpA[i], n = rpA[i + 1] - a, o = rp[i];
    for (int64_t q = lane_id(); q < n; q += WAVE) {
      col[o + q] = cA[a + q];
      val[o + q] = vA[a + q];
    }
    if (lane_id() == 0) {
      col[o + n] = (int32_t)(k + i);  // after every column of A: the row stays ascending
      val[o + n] = one;
    }
  }
}

__global__ void aug_b_rowptr(const int64_t *__restrict__ rpB, int64_t k, const int64_t *__restrict__ rpC, int64_t m,
                             int64_t *__restrict__ rp) {
  const int64_t b0 = rpB[0], nb = rpB[k] - b0, c0 = rpC[0];
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= k + m; r += (int64_t)gridDim.x * blockDim.x)
    rp[r] = r <= k ? rpB[r] - b0 : nb + (rpC[r - k] - c0);
}

template <class V>
__global__ void aug_b_entries(const int64_t *__restrict__ rpB, const int32_t *__restrict__ cB,
                              const V *__restrict__ vB, int64_t nb, const int64_t *__restrict__ rpC,
                              const int32_t *__restrict__ cC, const V *__restrict__ vC, int64_t nc,
                              int32_t *__restrict__ col, V *__restrict__ val) {
  const int64_t b0 = rpB[0], c0 = rpC[0];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nb + nc; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nb) {
      col[e] = cB[b0 + e];
      val[e] = vB[b0 + e];
    } else {
      col[e] = cC[c0 + e - nb];
      val[e] = vC[c0 + e - nb];
    }
  }
}

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

// The augmented operands of C_old (+) A (x) B; views into `keep`.
struct Augmented {
  Buf arp, acol, aval, brp, bcol, bval;
  CsrView a, b;
};

template <class V>
void augment_typed(Ctx *c, const CsrView &A, const CsrView &B, const CsrView &Cold, V one, Augmented *g,
                   hipStream_t s) {
  const int64_t m = A.m, k = A.n;
  const int64_t nA = A.nnz + m, nB = B.nnz + Cold.nnz;
  g->arp = Buf(c, sizeof(int64_t) * (size_t)(m + 1));
  g->acol = Buf(c, sizeof(int32_t) * (size_t)std::max<int64_t>(nA, 1));
  g->aval = Buf(c, sizeof(V) * (size_t)std::max<int64_t>(nA, 1));
  g->brp = Buf(c, sizeof(int64_t) * (size_t)(k + m + 1));
  g->bcol = Buf(c, sizeof(int32_t) * (size_t)std::max<int64_t>(nB, 1));
  g->bval = Buf(c, sizeof(V) * (size_t)std::max<int64_t>(nB, 1));
  aug_a_rowptr<<<grid_for(m + 1), 256, 0, s>>>(A.rowptr, m, g->arp.as<int64_t>());
  SRTC_LAUNCH_CHECK("aug_a_rowptr");
  aug_a_entries<V><<<grid_for(m * WAVE), 256, 0, s>>>(A.rowptr, A.col, (const V *)A.val, m, k, one,
                                                       g->arp.as<int64_t>(), g->acol.as<int32_t>(), g->aval.as<V>());
  SRTC_LAUNCH_CHECK("aug_a_entries");
  aug_b_rowptr<<<grid_for(k + m + 1), 256, 0, s>>>(B.rowptr, k, Cold.rowptr, m, g->brp.as<int64_t>());
  SRTC_LAUNCH_CHECK("aug_b_rowptr");
  if (nB > 0) {
    aug_b_entries<V><<<grid_for(nB), 256, 0, s>>>(B.rowptr, B.col, (const V *)B.val, B.nnz, Cold.rowptr, Cold.col,
                                                   (const V *)Cold.val, Cold.nnz, g->bcol.as<int32_t>(),
                                                   g->bval.as<V>());
    SRTC_LAUNCH_CHECK("aug_b_entries");
  }
  g->a = CsrView{m, k + m, nA, g->arp.as<int64_t>(), g->acol.as<int32_t>(), g->aval.p};
  g->b = CsrView{k + m, B.n, nB, g->brp.as<int64_t>(), g->bcol.as<int32_t>(), g->bval.p};
}

void augment(Ctx *c, int sr, int dt, const CsrView &A, const CsrView &B, const CsrView &Cold, Augmented *g,
             hipStream_t s) {
  // the multiplicative identity of each semiring (Section 3.1)
  switch (dt) {
    case SRTC_F64: augment_typed<double>(c, A, B, Cold, 1.0, g, s); break;
    case SRTC_F32: augment_typed<float>(c, A, B, Cold, sr == SRTC_MIN_PLUS ? 0.f : 1.f, g, s); break;
    case SRTC_I32: augment_typed<int32_t>(c, A, B, Cold, 0, g, s); break;
    case SRTC_BOOL8: augment_typed<uint8_t>(c, A, B, Cold, (uint8_t)1, g, s); break;
    case SRTC_PATH64: augment_typed<uint64_t>(c, A, B, Cold, (uint64_t)0, g, s); break;
    default: fail(SRTC_ERR_DTYPE, "accumulate: value type");
  }
}

}  // namespace

IdVal make_id_public(int sr, int dt, const void *add_id) { return make_id(sr, dt, add_id); }

// The schedule of an SpGEMM: a forced one (the argument, else the
// environment's SRTC_FORCE_SCHEDULE), else the autotune cache's entry for
// the problem's features, else the learned selector's pick, else schedule 0.
int choose_schedule(srtc_ctx *ctx, int sr, int dt, const CsrView &A, const CsrView &B, int requested,
                    hipStream_t s) {
  Ctx *c = &ctx->c;
  if (requested >= SRTC_NUM_SCHEDULES) fail(SRTC_ERR_ARG, "schedule id out of range");
  if (requested >= 0) return requested;
  if (c->force_schedule >= 0) return c->force_schedule;
  int sched = 0;
  if (c->mlp || !c->tune_cache.empty()) {
    float feat[SRTC_NUM_FEATURES];
    spgemm_features(c, sr, dt, A, B, feat, s);
    auto hit = c->tune_cache.find(tune_key(sr, dt, feat));
    int32_t pick = 0;
    if (hit != c->tune_cache.end()) sched = hit->second;
    else if (c->mlp && srtc_select(ctx, feat, &pick) == SRTC_OK) sched = pick;
    c->tracef("schedule: %d (%s)", sched, hit != c->tune_cache.end() ? "autotune cache" : "selector");
  }
  return sched;
}

std::string tune_key(int sr, int dt, const float *f) {
  std::string k = std::to_string(sr) + ":" + std::to_string(dt);
  char buf[32];
  for (int q = 0; q < SRTC_NUM_FEATURES; q++) {
    snprintf(buf, sizeof(buf), ":%.3g", (double)f[q]);
    k += buf;
  }
  return k;
}

}  // namespace srtc

using namespace srtc;

extern "C" {

const char *srtc_status_string(srtc_status st) {
  switch (st) {
    case SRTC_OK: return "ok";
    case SRTC_ERR_ARG: return "invalid argument";
    case SRTC_ERR_INDEX: return "invalid index string";
    case SRTC_ERR_DIM: return "dimension mismatch";
    case SRTC_ERR_DTYPE: return "value type not defined for the semiring";
    case SRTC_ERR_FORMAT: return "malformed sparse operand";
    case SRTC_ERR_ALIAS: return "output overlaps an input";
    case SRTC_ERR_OOM: return "out of memory";
    case SRTC_ERR_NOT_CONVERGED: return "fixpoint not reached";
    case SRTC_ERR_UNSUPPORTED: return "unsupported";
    case SRTC_ERR_DEVICE: return "device error";
    case SRTC_ERR_TOO_LARGE: return "request exceeds a fixed-size buffer";
  }
  return "unknown status";
}

srtc_status srtc_ctx_create(int device, srtc_alloc_fn alloc, srtc_free_fn free_fn, void *user, srtc_ctx **out) {
  if (!out) return SRTC_ERR_ARG;
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) return SRTC_ERR_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SRTC_ERR_DEVICE;
  srtc_ctx *c = new (std::nothrow) srtc_ctx();
  if (!c) return SRTC_ERR_OOM;
  c->c.device = device;
  c->c.alloc = alloc;
  c->c.free_fn = free_fn;
  c->c.user = user;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->c.num_cus = prop.multiProcessorCount;
    c->c.lds_per_block = prop.sharedMemPerBlock;
  }
  {
    // the fixed buffer of srtc_contract_noalloc: its address on this device,
    // looked up once per device with the device current
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) {
      delete c;
      return SRTC_ERR_DEVICE;
    }
    srtc_status st = SRTC_OK;
    try {
      c->c.fixed_scratch = spmm_fixed_scratch_init(device);
    } catch (const Error &e) {
      st = e.st;
    }
    (void)hipSetDevice(prev);
    if (st != SRTC_OK) {
      delete c;
      return st;
    }
  }
  const char *tr = getenv("SRTC_TRACE");
  c->c.trace = tr && *tr && *tr != '0';
  const char *va = getenv("SRTC_VALIDATE");
  c->c.validate_all = va && *va && *va != '0';
  const char *fs = getenv("SRTC_FORCE_SCHEDULE");
  if (fs && *fs) {
    char *end = nullptr;
    const long v = strtol(fs, &end, 10);
    if (end == fs || *end != 0 || v < 0 || v >= SRTC_NUM_SCHEDULES) {
      delete c;
      return SRTC_ERR_ARG;
    }
    c->c.force_schedule = (int)v;
  }
  const char *cb = getenv("SRTC_COL_BLOCKS");
  if (cb && *cb) {
    char *end = nullptr;
    const long v = strtol(cb, &end, 10);
    if (end == cb || *end != 0 || v < 0 || v > 4096) {
      delete c;
      return SRTC_ERR_ARG;
    }
    c->c.col_blocks = (int)v;
  }
  const char *ht = getenv("SRTC_HUB_TILE");
  if (ht && *ht) {
    char *end = nullptr;
    const long v = strtol(ht, &end, 10);
    if (end == ht || *end != 0 || v < 0 || v > 16384) {
      delete c;
      return SRTC_ERR_ARG;
    }
    c->c.hub_tile = (int)v;
  }
  const char *lb = getenv("SRTC_LDS_BUDGET");
  if (lb && *lb) {
    char *end = nullptr;
    const long long v = strtoll(lb, &end, 10);
    if (end == lb || *end != 0 || v < 16384) {
      delete c;
      return SRTC_ERR_ARG;
    }
    c->c.lds_budget = (int64_t)v;
  }
  *out = c;
  return SRTC_OK;
}

srtc_status srtc_profile_enable(srtc_ctx *ctx, int32_t on) {
  return guard(ctx, [&] {
    ctx->c.prof_resolve();
    ctx->c.prof.clear();
    ctx->c.profiling = on != 0;
  });
}

srtc_status srtc_profile_query(srtc_ctx *ctx, int32_t idx, char *name, int32_t name_len, int64_t *launches,
                               double *total_ms, double *total_bytes) {
  return guard(ctx, [&] {
    ctx->c.prof_resolve();
    if (idx < 0 || idx >= (int32_t)ctx->c.prof.size()) fail(SRTC_ERR_ARG, "no such profile entry");
    const Ctx::ProfAgg &a = ctx->c.prof[idx];
    if (name && name_len > 0) {
      strncpy(name, a.name.c_str(), (size_t)name_len - 1);
      name[name_len - 1] = 0;
    }
    if (launches) *launches = a.launches;
    if (total_ms) *total_ms = a.ms;
    if (total_bytes) *total_bytes = a.bytes;
  });
}

srtc_status srtc_ctx_destroy(srtc_ctx *ctx) {
  if (!ctx) return SRTC_ERR_ARG;
  try { ctx->c.prof_resolve(); } catch (...) {}
  for (auto e : ctx->c.event_pool) (void)hipEventDestroy(e);
  ctx->c.release_cache();
  if (ctx->c.pinned) (void)hipHostFree(ctx->c.pinned);
  mlp_destroy(ctx->c.mlp);
  delete ctx;
  return SRTC_OK;
}

const char *srtc_last_error(const srtc_ctx *ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

srtc_status srtc_fold(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, const char *isrc, const srtc_tensor *src,
                      const char *rows, const char *cols, srtc_tensor *out, void *stream) {
  return guard(ctx, [&] {
    check_tensor(src, "src");
    if (!out) fail(SRTC_ERR_ARG, "out: null");
    if (src->format == SRTC_DENSE) fail(SRTC_ERR_UNSUPPORTED, "fold takes a sparse (COO/CSR) tensor");
    const std::string idx = letters(isrc, src, "src");
    if (!rows || !cols) fail(SRTC_ERR_INDEX, "null row/col string");
    const std::string r(rows), cl(cols);
    std::string all = r + cl;
    if (all.size() != idx.size()) fail(SRTC_ERR_INDEX, "rows+cols must name every source index once");
    for (char ch : all)
      if (idx.find(ch) == std::string::npos || std::count(all.begin(), all.end(), ch) != 1)
        fail(SRTC_ERR_INDEX, "rows+cols must name every source index once");
    const IdVal id = make_id(sr, src->dtype, add_id);
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    ctx->c.tracef("srtc_fold %s -> (%s)(%s), %lld entries", idx.c_str(), r.c_str(), cl.c_str(), (long long)src->nnz);
    Folded f;
    fold_sparse(&ctx->c, sr, id, src, idx, r, cl, &f, s, true);
    int64_t dims[SRTC_MAX_ORDER];
    for (size_t q = 0; q < all.size(); q++) dims[q] = src->dims[idx.find(all[q])];
    set_csr_out(out, f.own, (int)all.size(), dims, (int)r.size(), src->dtype);
  });
}

srtc_status srtc_contract(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, int accumulate, const char *ia,
                          const srtc_tensor *A, const char *ib, const srtc_tensor *B, const char *ic, srtc_tensor *C,
                          const srtc_opts *opts, void *stream) {
  return guard(ctx, [&] {
    check_tensor(A, "A");
    check_tensor(B, "B");
    if (!C) fail(SRTC_ERR_ARG, "C: null");
    if (C->order < 0 || C->order > SRTC_MAX_ORDER) fail(SRTC_ERR_ARG, "C: bad order");
    const std::string a = letters(ia, A, "A"), b = letters(ib, B, "B"), cidx = letters(ic, C, "C");
    if (A->dtype != B->dtype) fail(SRTC_ERR_DTYPE, "A and B value types differ");
    const int dt = A->dtype;
    const IdVal id = make_id(sr, dt, add_id);
    const Plan p = plan_contraction(a, A, b, B, cidx, C);
    srtc_opts o{-1, 1, 0, 0};
    if (opts) o = *opts;
    if (o.hub_tile < 0 || o.hub_tile > 16384) fail(SRTC_ERR_ARG, "opts.hub_tile out of range (0..16384)");
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    Ctx *c = &ctx->c;
    c->tracef("srtc_contract %s,%s->%s semiring %d dtype %d", a.c_str(), b.c_str(), cidx.c_str(), (int)sr, dt);
    const std::string crow = rows_of_c(cidx, p);  // batch + M letters in C order
    std::string acol = p.batch, brow = p.batch, bcol = p.batch;
    acol += p.K;
    brow += p.K;
    bcol += p.N;
    const bool a_sparse = A->format != SRTC_DENSE, b_sparse = B->format != SRTC_DENSE;
    if (o.validate || c->validate_all) {
      validate_operand(c, sr, A, "A", s, &id);
      validate_operand(c, sr, B, "B", s, &id);
      if (accumulate && C->format == SRTC_CSR) validate_operand(c, sr, C, "C", s, &id);
    }
    if (a_sparse && b_sparse) {
      if (C->format == SRTC_DENSE) fail(SRTC_ERR_UNSUPPORTED, "sparse x sparse gives a sparse (CSR) C");
      Folded fa, fb;
      fold_sparse(c, sr, id, A, a, crow, acol, &fa, s);
      fold_sparse(c, sr, id, B, b, brow, bcol, &fb, s);
      const int sched = choose_schedule(ctx, sr, dt, fa.view, fb.view, o.schedule, s);
      CsrOut t;
      SpgemmStats st;
      // += without batch letters or a fold-back: the old C joins the
      // product's accumulators directly (one product, no merge pass)
      const bool seeded = accumulate && C->format == SRTC_CSR && C->nnz > 0 && p.batch.empty() &&
                          crow + p.N == cidx && fa.view.n + fa.view.m < 0x7fffffff;
      if (seeded) {
        if (C->split != (int)crow.size()) fail(SRTC_ERR_FORMAT, "C: split differs from the row indices");
        if (C->dtype != dt) fail(SRTC_ERR_DTYPE, "C value type differs");
        CsrView cv = csr_view(C);
        if (cv.m != fa.view.m || cv.n != fb.view.n) fail(SRTC_ERR_DIM, "C: shape differs from the product's");
        if (fa.view.n != fb.view.m) fail(SRTC_ERR_DIM, "inner dimensions differ");
        Augmented g;
        augment(c, sr, dt, fa.view, fb.view, cv, &g, s);
        spgemm(c, sr, dt, id, g.a, g.b, sched, o.sorted, &t, &st, s);
        int64_t dims[SRTC_MAX_ORDER];
        for (size_t q = 0; q < cidx.size(); q++) dims[q] = p.dim.at(cidx[q]);
        set_csr_out(C, t, (int)cidx.size(), dims, (int)crow.size(), dt);
        return;
      }
      const int64_t hub = o.hub_tile > 0 ? o.hub_tile : c->hub_tile;
      const bool merge_old = accumulate && C->format == SRTC_CSR && C->nnz > 0;
      if (!merge_old && p.batch.empty() && crow + p.N == cidx && hub_product_applies(sr, dt, fa.view, fb.view, hub)) {
        if (fa.view.n != fb.view.m) fail(SRTC_ERR_DIM, "inner dimensions differ");
        spgemm_hubs(c, dt, id, fa.view, fb.view, hub, sched, o.sorted, &t, &st, s);
        int64_t dims[SRTC_MAX_ORDER];
        for (size_t q = 0; q < cidx.size(); q++) dims[q] = p.dim.at(cidx[q]);
        set_csr_out(C, t, (int)cidx.size(), dims, (int)crow.size(), dt);
        return;
      }
      spgemm(c, sr, dt, id, fa.view, fb.view, sched, o.sorted, &t, &st, s);
      if (!p.batch.empty() && t.nnz > 0) {
        col_mod_kernel<<<4096, 256, 0, s>>>(t.col.as<int32_t>(), t.nnz, extent(p, p.N));
        SRTC_LAUNCH_CHECK("col_mod_kernel");
      }
      t.n = extent(p, p.N);
      if (crow + p.N != cidx && t.nnz > 0) {
        // fold back: the product's (C's row letters) x (C's column letters)
        // entries become C in its own index order, rows = C's first
        // |rows| letters (a permutation of keys, so nothing combines)
        const std::string from = crow + p.N;
        std::vector<int64_t> fd(from.size());
        for (size_t q = 0; q < from.size(); q++) fd[q] = p.dim.at(from[q]);
        std::vector<int> rm, cm;
        for (size_t q = 0; q < cidx.size(); q++)
          (q < crow.size() ? rm : cm).push_back((int)from.find(cidx[q]));
        CsrView tv{t.m, t.n, t.nnz, t.rowptr.as<int64_t>(), t.col.as<int32_t>(), t.val.p};
        Buf k0(c, sizeof(int64_t) * (size_t)t.nnz), k1(c, sizeof(int64_t) * (size_t)t.nnz);
        csr_to_keys(tv, k0.as<int64_t>(), s);
        remap_keys(c, k0.as<int64_t>(), t.nnz, (int)from.size(), fd.data(), (int)rm.size(), rm.data(), (int)cm.size(),
                   cm.data(), k1.as<int64_t>(), s);
        int64_t nr = 1, nc = 1;
        for (int q : rm) nr *= fd[q];
        for (int q : cm) nc *= fd[q];
        CsrOut u;
        fold_keys_to_csr(c, sr, dt, id, k1.as<int64_t>(), t.val.p, t.nnz, nr, nc, &u, s);
        t = std::move(u);
      }
      if (accumulate && C->format == SRTC_CSR && C->nnz > 0) {
        // previous C joins the sum: C_new = C_old (+) T (old entries first)
        if (C->split != (int)crow.size()) fail(SRTC_ERR_FORMAT, "C: split differs from the row indices");
        CsrView cv = csr_view(C);
        CsrView tv{t.m, t.n, t.nnz, t.rowptr.as<int64_t>(), t.col.as<int32_t>(), t.val.p};
        CsrOut u;
        ewise_add(c, sr, dt, id, cv, tv, &u, s);
        t = std::move(u);
      }
      int64_t dims[SRTC_MAX_ORDER];
      for (size_t q = 0; q < cidx.size(); q++) dims[q] = p.dim.at(cidx[q]);
      set_csr_out(C, t, (int)cidx.size(), dims, (int)crow.size(), dt);
      return;
    }
    if (C->format != SRTC_DENSE) fail(SRTC_ERR_UNSUPPORTED, "a dense operand gives a dense C");
    if (C->dtype != dt) fail(SRTC_ERR_DTYPE, "C value type differs");
    if (!C->vals) fail(SRTC_ERR_ARG, "C: no values");
    const size_t cbytes = tensor_value_bytes(C);
    if (overlaps(C->vals, cbytes, A->vals, tensor_value_bytes(A)) ||
        overlaps(C->vals, cbytes, B->vals, tensor_value_bytes(B)))
      fail(SRTC_ERR_ALIAS, "C overlaps an operand");
    // dense B must be laid out as (batch, K) rows x N columns
    auto dense_in_order = [&](const srtc_tensor *T, const std::string &idx, const std::string &want, Buf *tmp)
        -> const void * {
      if (idx == want) return T->vals;
      std::vector<int> perm;
      for (char ch : want) perm.push_back((int)idx.find(ch));
      *tmp = Buf(c, tensor_value_bytes(T));
      dense_permute(T->vals, tmp->p, (int)dtype_size(dt), T->order, T->dims, perm.data(), s);
      return tmp->p;
    };
    // The product is formed in the order `from` of its own rows and
    // columns; when that is not C's order it goes to a scratch tensor and
    // is folded back (permuted, the old C joining by (+) with accumulate).
    auto product_into_c = [&](const std::string &from, auto &&form) {
      if (from == cidx) {
        form(C->vals, accumulate);
        return;
      }
      Buf tc(c, cbytes);
      form(tc.p, 0);
      std::vector<int64_t> fd(from.size());
      for (size_t q = 0; q < from.size(); q++) fd[q] = p.dim.at(from[q]);
      std::vector<int> perm;
      for (char ch : cidx) perm.push_back((int)from.find(ch));
      ProfScope ps(c, "dense.fold_back", (accumulate ? 3.0 : 2.0) * (double)cbytes, s);
      if (accumulate)
        dense_permute_combine(sr, dt, id, tc.p, C->vals, (int)from.size(), fd.data(), perm.data(), s);
      else
        dense_permute(tc.p, C->vals, (int)dtype_size(dt), (int)from.size(), fd.data(), perm.data(), s);
    };
    if (a_sparse && !b_sparse) {
      Folded fa;
      fold_sparse(c, sr, id, A, a, crow, acol, &fa, s);
      Buf tb;
      const void *Bd = dense_in_order(B, b, brow + p.N, &tb);
      product_into_c(crow + p.N, [&](void *out, int acc) {
        spmm(c, sr, dt, id, fa.view, Bd, extent(p, p.N), out, acc, s);
      });
      return;
    }
    if (!a_sparse && !b_sparse && p.M.empty() && p.N.empty() && p.K.empty()) {
      // every letter in all three tensors: the elementwise product, any semiring
      Buf ta, tb;
      const void *Ad = dense_in_order(A, a, cidx, &ta);
      const void *Bd = dense_in_order(B, b, cidx, &tb);
      ProfScope ps(c, "dense.hadamard", (accumulate ? 4.0 : 3.0) * (double)cbytes, s);
      dense_hadamard(sr, dt, id, Ad, Bd, C->vals, prod_dims(C), accumulate, s);
      return;
    }
    if (!a_sparse && !b_sparse) {
      if (sr != SRTC_PLUS_TIMES) fail(SRTC_ERR_UNSUPPORTED, "dense x dense is defined for (+,x) only");
      // batched GEMM over (batch, M, K) x (batch, K, N) -> (batch, M, N)
      Buf ta, tb;
      const void *Ad = dense_in_order(A, a, p.batch + p.M + p.K, &ta);
      const void *Bd = dense_in_order(B, b, p.batch + p.K + p.N, &tb);
      const int64_t M_ = extent(p, p.M), N_ = extent(p, p.N), K_ = extent(p, p.K), Z_ = extent(p, p.batch);
      product_into_c(p.batch + p.M + p.N, [&](void *out, int acc) {
        const double es = (double)dtype_size(dt);
        ProfScope ps(c, dt == SRTC_F64 ? "dense.gemm_mfma.f64" : "dense.gemm_mfma.f32",
                     es * (double)Z_ * ((double)M_ * K_ + (double)K_ * N_ + (double)M_ * N_ * (acc ? 2 : 1)), s);
        dense_gemm_plus_times(c, dt, Ad, Bd, out, M_, N_, K_, acc, s, Z_);
      });
      return;
    }
    fail(SRTC_ERR_UNSUPPORTED, "dense A with sparse B: swap the operands");
  });
}

srtc_status srtc_contract_panels(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, const char *ia,
                                 const srtc_tensor *A, const char *ib, const srtc_tensor *B, const char *ic,
                                 const srtc_opts *opts, int64_t panel_products, srtc_panel_fn consume, void *user,
                                 void *stream) {
  return guard(ctx, [&] {
    check_tensor(A, "A");
    check_tensor(B, "B");
    if (!consume) fail(SRTC_ERR_ARG, "panels: null consumer");
    if (A->format == SRTC_DENSE || B->format == SRTC_DENSE)
      fail(SRTC_ERR_UNSUPPORTED, "panels: A and B must be sparse (COO or CSR)");
    const std::string a = letters(ia, A, "A"), b = letters(ib, B, "B");
    if (!ic) fail(SRTC_ERR_INDEX, "C: null index string");
    // C's extents come from the letters it shares with A and B
    srtc_tensor Ct{};
    Ct.order = (int32_t)strlen(ic);
    if (Ct.order > SRTC_MAX_ORDER) fail(SRTC_ERR_INDEX, "C: too many indices");
    for (int q = 0; q < Ct.order; q++) {
      const size_t pa = a.find(ic[q]), pb = b.find(ic[q]);
      Ct.dims[q] = pa != std::string::npos ? A->dims[pa] : pb != std::string::npos ? B->dims[pb] : 1;
    }
    const std::string cidx = letters(ic, &Ct, "C");
    if (A->dtype != B->dtype) fail(SRTC_ERR_DTYPE, "A and B value types differ");
    const int dt = A->dtype;
    const IdVal id = make_id(sr, dt, add_id);
    const Plan p = plan_contraction(a, A, b, B, cidx, &Ct);
    if (!p.batch.empty()) fail(SRTC_ERR_UNSUPPORTED, "panels: no index may appear in A, B and C");
    const std::string crow = rows_of_c(cidx, p);
    if (crow + p.N != cidx) fail(SRTC_ERR_UNSUPPORTED, "panels: C's row indices must precede its column indices");
    srtc_opts o{-1, 1, 0, 0};
    if (opts) o = *opts;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    Ctx *c = &ctx->c;
    if (o.validate || c->validate_all) {
      validate_operand(c, sr, A, "A", s, &id);
      validate_operand(c, sr, B, "B", s, &id);
    }
    Folded fa, fb;
    fold_sparse(c, sr, id, A, a, crow, p.K, &fa, s);
    fold_sparse(c, sr, id, B, b, p.K, p.N, &fb, s);
    const CsrView &av = fa.view;
    // one schedule for the whole product, from the features of all rows
    const int sched = choose_schedule(ctx, sr, dt, av, fb.view, o.schedule, s);
    const int64_t m = av.m;
    if (panel_products <= 0) panel_products = (int64_t)1 << 31;
    // panel cuts at running product counts
    std::vector<int64_t> pre((size_t)m + 1, 0), hrp((size_t)m + 1, 0);
    if (m > 0) {
      Buf w(c, sizeof(int64_t) * (size_t)m), wp(c, sizeof(int64_t) * (size_t)(m + 1));
      row_products(av, fb.view, w.as<int64_t>(), s);
      excl_scan_i64(c, w.as<int64_t>(), wp.as<int64_t>(), m, s);
      read_to_host(c, pre.data(), wp.p, sizeof(int64_t) * (size_t)(m + 1), s);
      read_to_host(c, hrp.data(), av.rowptr, sizeof(int64_t) * (size_t)(m + 1), s);
    }
    int64_t dims[2] = {m, fb.view.n};
    // B's window tables and value records are built for the first panel and
    // kept for the others (fb stays allocated and unchanged until the end)
    struct KeepB {
      Ctx *c;
      KeepB(Ctx *cc, const CsrView &b) : c(cc) { c->keep_b = Ctx::KeptB{b.rowptr, b.col, b.val, b.m, b.n, b.nnz}; }
      ~KeepB() {
        c->keep_b = Ctx::KeptB{};
        c->b_tables.clear();
      }
    } keep(c, fb.view);
    c->tracef("srtc_contract_panels: %lld rows, %lld products, schedule %d, at most %lld products per panel",
              (long long)m, (long long)pre[m], sched, (long long)panel_products);
    int64_t r0 = 0;
    while (r0 < m) {
      // the longest run of rows from r0 within the budget (at least one row)
      int64_t r1 = (int64_t)(std::upper_bound(pre.begin() + r0 + 1, pre.end(), pre[r0] + panel_products) - pre.begin()) - 1;
      if (r1 <= r0) r1 = r0 + 1;
      CsrView pv{r1 - r0, av.n, hrp[r1] - hrp[r0], av.rowptr + r0, av.col, av.val};
      CsrOut t;
      spgemm(c, sr, dt, id, pv, fb.view, sched, o.sorted, &t, nullptr, s);
      srtc_tensor Cp{};
      dims[0] = r1 - r0;
      set_csr_out(&Cp, t, 2, dims, 1, dt);
      const int32_t rc = consume(user, r0, r1 - r0, &Cp, stream);
      if (rc != 0) fail(SRTC_ERR_ARG, "panels: stopped by the consumer");
      r0 = r1;
    }
  });
}

srtc_status srtc_contract_noalloc(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, int accumulate,
                                  const char *ia, const srtc_tensor *A, const char *ib, const srtc_tensor *B,
                                  const char *ic, srtc_tensor *C, void *stream) {
  return guard(ctx, [&] {
    check_tensor(A, "A");
    check_tensor(B, "B");
    check_tensor(C, "C");
    const std::string a = letters(ia, A, "A"), b = letters(ib, B, "B"), cidx = letters(ic, C, "C");
    if (A->dtype != B->dtype) fail(SRTC_ERR_DTYPE, "A and B value types differ");
    const int dt = A->dtype;
    const IdVal id = make_id(sr, dt, add_id);
    const Plan p = plan_contraction(a, A, b, B, cidx, C);
    if (A->format != SRTC_CSR || B->format != SRTC_DENSE || C->format != SRTC_DENSE)
      fail(SRTC_ERR_UNSUPPORTED, "no-allocation contraction: A must be CSR, B and C dense");
    if (!p.batch.empty()) fail(SRTC_ERR_UNSUPPORTED, "no-allocation contraction: a letter in all three tensors");
    if (a != p.M + p.K || A->split != (int)p.M.size())
      fail(SRTC_ERR_UNSUPPORTED, "no-allocation contraction: A must be CSR over C's row letters then the inner ones");
    if (b != p.K + p.N) fail(SRTC_ERR_UNSUPPORTED, "no-allocation contraction: B must list A's inner letters first");
    if (cidx != p.M + p.N) fail(SRTC_ERR_UNSUPPORTED, "no-allocation contraction: C must list its row letters first");
    if (C->dtype != dt) fail(SRTC_ERR_DTYPE, "C value type differs");
    const size_t cbytes = tensor_value_bytes(C);
    if (overlaps(C->vals, cbytes, A->vals, tensor_value_bytes(A)) ||
        overlaps(C->vals, cbytes, B->vals, tensor_value_bytes(B)))
      fail(SRTC_ERR_ALIAS, "C overlaps an operand");
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    ctx->c.tracef("srtc_contract_noalloc %s,%s->%s semiring %d dtype %d", a.c_str(), b.c_str(), cidx.c_str(), (int)sr,
                  dt);
    spmm_fixed(&ctx->c, sr, dt, id, csr_view(A), B->vals, extent(p, p.N), C->vals, accumulate ? 1 : 0, s);
  });
}

srtc_status srtc_contract_masked(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, const char *ia,
                                 const srtc_tensor *A, const char *ib, const srtc_tensor *B, const char *ic,
                                 const srtc_tensor *M, srtc_tensor *C, const srtc_opts *opts, void *stream) {
  return guard(ctx, [&] {
    check_tensor(A, "A");
    check_tensor(B, "B");
    check_tensor(M, "M");
    if (!C) fail(SRTC_ERR_ARG, "C: null");
    if (C->order < 0 || C->order > SRTC_MAX_ORDER) fail(SRTC_ERR_ARG, "C: bad order");
    if (A->format == SRTC_DENSE || B->format == SRTC_DENSE || M->format == SRTC_DENSE)
      fail(SRTC_ERR_UNSUPPORTED, "masked contraction: A, B and the mask must be sparse");
    const std::string a = letters(ia, A, "A"), b = letters(ib, B, "B"), cidx = letters(ic, C, "C");
    const std::string midx = letters(ic, M, "M");
    if (A->dtype != B->dtype) fail(SRTC_ERR_DTYPE, "A and B value types differ");
    const int dt = A->dtype;
    const IdVal id = make_id(sr, dt, add_id);
    const Plan p = plan_contraction(a, A, b, B, cidx, C);
    if (!p.batch.empty()) fail(SRTC_ERR_UNSUPPORTED, "masked contraction: no index may appear in A, B and C");
    if (rows_of_c(cidx, p) + p.N != cidx)
      fail(SRTC_ERR_UNSUPPORTED, "masked contraction: C's index order interleaves row and column indices");
    for (size_t q = 0; q < cidx.size(); q++)
      if (M->dims[q] != p.dim.at(cidx[q])) fail(SRTC_ERR_DIM, "M: extents differ from C's");
    srtc_opts o{-1, 1, 0, 0};
    if (opts) o = *opts;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    Ctx *c = &ctx->c;
    if (o.validate || c->validate_all) {
      validate_operand(c, sr, A, "A", s, &id);
      validate_operand(c, sr, B, "B", s, &id);
      validate_operand(c, SRTC_OR_AND, M, "M", s);
    }
    const std::string crow = rows_of_c(cidx, p);
    const std::string acol = p.K, brow = p.K, bcol = p.N;
    Folded fa, fb, fm;
    fold_sparse(c, sr, id, A, a, crow, acol, &fa, s);
    fold_sparse(c, sr, id, B, b, brow, bcol, &fb, s);
    // the mask's values are ignored: fold it as a pattern (duplicates merge)
    srtc_tensor mp = *M;
    const IdVal mid = make_id(SRTC_OR_AND, SRTC_BOOL8, nullptr);
    Buf ones(c, (size_t)std::max<int64_t>(M->nnz, 1));
    fill_bytes_value(ones.p, std::max<int64_t>(M->nnz, 1), SRTC_BOOL8, IdVal{1.0, 1}, s);
    mp.vals = ones.p;
    mp.dtype = SRTC_BOOL8;
    fold_sparse(c, SRTC_OR_AND, mid, &mp, midx, crow, bcol, &fm, s);
    c->tracef("srtc_contract_masked %s,%s->%s semiring %d dtype %d, mask nnz %lld", a.c_str(), b.c_str(),
              cidx.c_str(), (int)sr, dt, (long long)fm.view.nnz);
    CsrOut t;
    spgemm_masked(c, sr, dt, id, fa.view, fb.view, fm.view, &t, s);
    int64_t dims[SRTC_MAX_ORDER];
    for (size_t q = 0; q < cidx.size(); q++) dims[q] = p.dim.at(cidx[q]);
    set_csr_out(C, t, (int)cidx.size(), dims, (int)crow.size(), dt);
  });
}

srtc_status srtc_fixpoint(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, const srtc_tensor *A, srtc_tensor *X,
                          int64_t max_iters, int32_t steps_per_check, int64_t *iters_out, void *stream) {
  return srtc_fixpoint_ex(ctx, sr, add_id, A, X, max_iters, steps_per_check, 0, iters_out, stream);
}

srtc_status srtc_fixpoint_ex(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, const srtc_tensor *A,
                             srtc_tensor *X, int64_t max_iters, int32_t steps_per_check, int32_t flags,
                             int64_t *iters_out, void *stream) {
  return guard(ctx, [&] {
    if (flags & ~SRTC_FIXPOINT_CHANGED_ROWS) fail(SRTC_ERR_ARG, "unknown fixpoint flags");
    check_tensor(A, "A");
    check_tensor(X, "X");
    if (A->format != SRTC_CSR || A->order != 2 || A->split != 1) fail(SRTC_ERR_FORMAT, "A must be a CSR matrix");
    if (X->format != SRTC_DENSE || X->order < 1 || X->order > 2) fail(SRTC_ERR_FORMAT, "X must be a dense n or n x s array");
    if (sr == SRTC_PLUS_TIMES) fail(SRTC_ERR_UNSUPPORTED, "fixpoint needs an idempotent semiring");
    if (A->dtype != X->dtype) fail(SRTC_ERR_DTYPE, "A and X value types differ");
    const int dt = A->dtype;
    const IdVal id = make_id(sr, dt, add_id);
    const int64_t n = A->dims[0];
    if (A->dims[1] != n || X->dims[0] != n) fail(SRTC_ERR_DIM, "A must be n x n and X n x s");
    const int64_t sw = X->order == 2 ? X->dims[1] : 1;
    if (max_iters <= 0) max_iters = n;
    int k = std::max(2, (int)steps_per_check);
    if (k % 2) k++;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    Ctx *c = &ctx->c;
    CsrView av = csr_view(A);
    SpmmPlan pl;
    pl.build(c, av, sw, s);
    const size_t bytes = tensor_value_bytes(X);
    Buf xb(c, bytes);
    Buf chg(c, sizeof(int32_t) * (size_t)k);  // one change flag per step
    void *xa = X->vals;
    void *bufs[2] = {xa, xb.p};
    // changed-row masks, double-buffered like X: step t reads rch[t&1] and
    // writes rch[(t&1)^1]; cleared by a fill kernel (graph-safe)
    const bool delta = (flags & SRTC_FIXPOINT_CHANGED_ROWS) != 0;
    const int64_t nw = (n + 3) / 4;  // int32 words per mask
    Buf rch;
    uint8_t *rbuf[2] = {nullptr, nullptr};
    if (delta) {
      rch = Buf(c, sizeof(int32_t) * (size_t)std::max<int64_t>(2 * nw, 1));
      rbuf[0] = rch.as<uint8_t>();
      rbuf[1] = rch.as<uint8_t>() + 4 * nw;
      fill_i32(reinterpret_cast<int32_t *>(rbuf[0]), nw, 0x01010101, s);  // first step: every row
    }
    auto step = [&](int t, int parity, hipStream_t st) {
      fill_i32(chg.as<int32_t>() + t, 1, 0, st);
      if (delta) fill_i32(reinterpret_cast<int32_t *>(rbuf[parity ^ 1]), nw, 0, st);
      spmm_with_plan(pl, sr, dt, id, av, bufs[parity], sw, bufs[parity ^ 1], 1, 0, chg.as<int32_t>() + t,
                     nullptr, nullptr, nullptr, st, delta ? rbuf[parity] : nullptr, delta ? rbuf[parity ^ 1] : nullptr);
    };
    // capture k steps (k even: the iterate returns to X)
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
    c->tracef("srtc_fixpoint n=%lld s=%lld, capturing %d steps", (long long)n, (long long)sw, k);
    SRTC_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    for (int t = 0; t < k; t++) step(t, t & 1, cap);
    SRTC_HIP(hipStreamEndCapture(cap, &graph));
    SRTC_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    std::vector<int32_t> hf(k);
    int64_t r = 0;
    while (r < max_iters) {
      int nsteps;
      if (r + k <= max_iters) {
        SRTC_HIP(hipGraphLaunch(exec, s));
        nsteps = k;
      } else {
        nsteps = (int)(max_iters - r);
        for (int t = 0; t < nsteps; t++) step(t, t & 1, s);
        if (nsteps & 1) SRTC_HIP(hipMemcpyAsync(xa, xb.p, bytes, hipMemcpyDeviceToDevice, s));
      }
      read_to_host(c, hf.data(), chg.p, sizeof(int32_t) * (size_t)nsteps, s);
      for (int t = 0; t < nsteps; t++) {
        if (hf[t] == 0) {
          if (iters_out) *iters_out = r + t + 1;
          return;
        }
      }
      r += nsteps;
    }
    if (iters_out) *iters_out = r;
    fail(SRTC_ERR_NOT_CONVERGED, "still changing after max_iters steps");
  });
}

srtc_status srtc_bfs_levels(srtc_ctx *ctx, const srtc_tensor *A, const int64_t *sources, int32_t nsrc, int32_t *levels,
                            int32_t *depth_out, void *stream) {
  return guard(ctx, [&] {
    check_tensor(A, "A");
    if (A->format != SRTC_CSR || A->order != 2 || A->split != 1) fail(SRTC_ERR_FORMAT, "A must be a CSR matrix");
    if (nsrc < 1 || nsrc > 64) fail(SRTC_ERR_ARG, "1..64 sources");
    if (!sources || !levels) fail(SRTC_ERR_ARG, "null sources/levels");
    const int64_t n = A->dims[0];
    if (A->dims[1] != n) fail(SRTC_ERR_DIM, "A must be square");
    for (int t = 0; t < nsrc; t++)
      if (sources[t] < 0 || sources[t] >= n) fail(SRTC_ERR_ARG, "source out of range");
    for (int t = 0; t < nsrc; t++)
      for (int u = t + 1; u < nsrc; u++)
        if (sources[t] == sources[u]) fail(SRTC_ERR_ARG, "repeated source");
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    Ctx *c = &ctx->c;
    CsrView av = csr_view(A);
    Buf fa(c, 8 * (size_t)n), fb(c, 8 * (size_t)n), vis(c, 8 * (size_t)n), src(c, 8 * 64), chg(c, 64);
    fill_i64((int64_t *)fa.p, n, 0, s);
    fill_i64((int64_t *)vis.p, n, 0, s);
    fill_i32(levels, n * nsrc, -1, s);
    int64_t *hs = (int64_t *)c->host_scratch(8 * 64);
    memcpy(hs, sources, 8 * (size_t)nsrc);
    SRTC_HIP(hipMemcpyAsync(src.p, hs, 8 * (size_t)nsrc, hipMemcpyHostToDevice, s));
    bfs_init<<<1, 64, 0, s>>>(src.as<int64_t>(), nsrc, fa.as<uint64_t>(), vis.as<uint64_t>(), levels);
    SRTC_LAUNCH_CHECK("bfs_init");
    uint64_t *cur = fa.as<uint64_t>(), *nxt = fb.as<uint64_t>();
    int32_t depth = 0;
    for (int level = 1; level <= n; level++) {
      fill_i32(chg.as<int32_t>(), 1, 0, s);
      {
        ProfScope ps(c, "bfs.step", 4.0 * av.nnz + 8.0 * (n + 1) + 24.0 * n, s);
        bfs_step(av, cur, vis.as<uint64_t>(), nxt, levels, nsrc, level, chg.as<int32_t>(), s);
      }
      int32_t h = 0;
      read_to_host(c, &h, chg.p, sizeof(int32_t), s);
      if (!h) break;
      depth = level;
      std::swap(cur, nxt);
    }
    if (depth_out) *depth_out = depth;
  });
}

srtc_status srtc_transform(srtc_ctx *ctx, srtc_transform_op op, double alpha, const char *ia, const srtc_tensor *A,
                           const char *ib, const srtc_tensor *B, const char *ic, srtc_tensor *C, void *stream) {
  return guard(ctx, [&] {
    if (op < SRTC_TF_RECIP || op > SRTC_TF_DIV_SUM) fail(SRTC_ERR_ARG, "unknown transform");
    check_tensor(C, "C");
    if (C->dtype != SRTC_F64 && C->dtype != SRTC_F32) fail(SRTC_ERR_DTYPE, "transforms are defined for F64 and F32");
    const bool need_a = op == SRTC_TF_ADD || op == SRTC_TF_FMA || op == SRTC_TF_DIV_SUM;
    const bool need_b = op == SRTC_TF_FMA || op == SRTC_TF_DIV_SUM;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    const std::string cidx = letters(ic, C, "C");
    int64_t zero = 0;
    if (C->format != SRTC_DENSE) {
      if (need_a || need_b) fail(SRTC_ERR_UNSUPPORTED, "a sparse C takes RECIP and SCALE only");
      int64_t nv = C->nnz;
      transform_dense_call(op, C->dtype, alpha, &nv, 1, nullptr, &zero, nullptr, &zero, C->vals, s);
      return;
    }
    const int order = C->order;
    std::vector<int64_t> ext(std::max(order, 1), 1), sa(std::max(order, 1), 0), sb(std::max(order, 1), 0);
    for (int q = 0; q < order; q++) ext[q] = C->dims[q];
    const size_t cbytes = tensor_value_bytes(C);
    auto strides = [&](const srtc_tensor *T, const char *idx, const char *name, std::vector<int64_t> &st) {
      check_tensor(T, name);
      if (T->format != SRTC_DENSE) fail(SRTC_ERR_FORMAT, std::string(name) + ": must be dense");
      if (T->dtype != C->dtype) fail(SRTC_ERR_DTYPE, std::string(name) + ": value type differs from C's");
      const std::string l = letters(idx, T, name);
      std::vector<int64_t> ts(T->order);
      int64_t acc = 1;
      for (int q = T->order - 1; q >= 0; q--) {
        ts[q] = acc;
        acc *= T->dims[q];
      }
      for (size_t q = 0; q < l.size(); q++) {
        const size_t pos = cidx.find(l[q]);
        if (pos == std::string::npos) fail(SRTC_ERR_INDEX, std::string(name) + ": a letter missing from C");
        if (T->dims[q] != C->dims[pos]) fail(SRTC_ERR_DIM, std::string(name) + ": extent differs from C's");
        st[pos] = ts[q];
      }
      if (overlaps(C->vals, cbytes, T->vals, tensor_value_bytes(T))) fail(SRTC_ERR_ALIAS, "C overlaps an operand");
      return (const void *)T->vals;
    };
    const void *Ap = need_a ? strides(A, ia, "A", sa) : nullptr;
    const void *Bp = need_b ? strides(B, ib, "B", sb) : nullptr;
    ProfScope ps(&ctx->c, "transform", 2.0 * (double)cbytes, s);
    transform_dense_call(op, C->dtype, alpha, ext.data(), order, Ap, sa.data(), Bp, sb.data(), C->vals, s);
  });
}

srtc_status srtc_jacobi(srtc_ctx *ctx, const srtc_tensor *A, const srtc_tensor *b, srtc_tensor *x, double tol,
                        int64_t max_iters, int32_t steps_per_check, int64_t *iters_out, double *resid_out,
                        void *stream) {
  return guard(ctx, [&] {
    check_tensor(A, "A");
    check_tensor(b, "b");
    check_tensor(x, "x");
    if (A->order != 2 || A->format == SRTC_DENSE) fail(SRTC_ERR_FORMAT, "A must be a sparse matrix (COO or CSR)");
    const int64_t n = A->dims[0];
    if (A->dims[1] != n) fail(SRTC_ERR_DIM, "A must be square");
    const int dt = A->dtype;
    if (dt != SRTC_F64 && dt != SRTC_F32) fail(SRTC_ERR_DTYPE, "Jacobi is defined for F64 and F32");
    for (const srtc_tensor *v : {b, (const srtc_tensor *)x}) {
      if (v->format != SRTC_DENSE || v->order != 1) fail(SRTC_ERR_FORMAT, "b and x must be dense vectors");
      if (v->dims[0] != n) fail(SRTC_ERR_DIM, "b and x must have n entries");
      if (v->dtype != dt) fail(SRTC_ERR_DTYPE, "b and x must have A's value type");
    }
    if (!(tol >= 0.0)) fail(SRTC_ERR_ARG, "tol must be >= 0");
    if (overlaps(x->vals, tensor_value_bytes(x), b->vals, tensor_value_bytes(b))) fail(SRTC_ERR_ALIAS, "x overlaps b");
    if (max_iters <= 0) max_iters = 10000;
    int k = std::max(2, (int)steps_per_check);
    if (k % 2) k++;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    Ctx *c = &ctx->c;
    Folded fa;
    fold_sparse(c, SRTC_PLUS_TIMES, IdVal{0.0, 0}, A, "ij", "i", "j", &fa, s);
    JacobiPlan pl;
    pl.build(c, dt, fa.view, s);
    const size_t bytes = dtype_size(dt) * (size_t)std::max<int64_t>(n, 1);
    Buf xb(c, bytes), stb(c, 64);
    fill_i32(stb.as<int32_t>(), 16, 0, s);  // iter = 0, not done
    JacobiState *st = reinterpret_cast<JacobiState *>(stb.p);
    void *bufs[2] = {x->vals, xb.p};
    const double tol2 = tol * tol;
    auto step = [&](int t, hipStream_t q) { jacobi_step_call(pl, b->vals, bufs[t & 1], bufs[(t & 1) ^ 1], st, tol2, q); };
    JacobiState hs{};
    if (n > 0) {
      // k steps per replay; after the stopping step the rest do nothing,
      // so x^l stays in buffer l & 1 (each replay has an even count)
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
      for (int t = 0; t < k; t++) step(t, cap);
      SRTC_HIP(hipStreamEndCapture(cap, &graph));
      SRTC_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      int64_t ran = 0;  // steps issued; the last one checks x^{ran-1}
      while (true) {
        if (ran + k <= max_iters + 1) {
          SRTC_HIP(hipGraphLaunch(exec, s));
          ran += k;
        } else {
          // the remaining steps one by one, parity continuing from `ran`
          const int64_t left = max_iters + 1 - ran;
          for (int64_t t = 0; t < left; t++) step((int)((ran + t) & 1), s);
          ran += left;
        }
        read_to_host(c, &hs, st, sizeof(hs), s);
        if (hs.done || ran >= max_iters + 1) break;
      }
      const int64_t l = hs.done ? hs.iter : max_iters;
      if (l & 1) SRTC_HIP(hipMemcpyAsync(x->vals, xb.p, bytes, hipMemcpyDeviceToDevice, s));
      if (iters_out) *iters_out = l;
      if (resid_out) *resid_out = std::sqrt(hs.rsq);
      if (!hs.done) fail(SRTC_ERR_NOT_CONVERGED, "residual above tol after max_iters updates");
    } else {
      if (iters_out) *iters_out = 0;
      if (resid_out) *resid_out = 0.0;
    }
  });
}

srtc_status srtc_apsp_tiskin(srtc_ctx *ctx, const void *add_id, const srtc_tensor *A, int32_t *D, int32_t *H,
                             int32_t *rounds_out, int64_t *round_nnz, void *stream) {
  return guard(ctx, [&] {
    check_tensor(A, "A");
    if (A->order != 2 || A->format == SRTC_DENSE) fail(SRTC_ERR_FORMAT, "A must be a sparse matrix (COO or CSR)");
    if (A->dtype != SRTC_I32) fail(SRTC_ERR_DTYPE, "apsp weights must be int32");
    const IdVal id = make_id(SRTC_MIN_PLUS, SRTC_I32, add_id);
    const int64_t n = A->dims[0];
    if (A->dims[1] != n) fail(SRTC_ERR_DIM, "A must be square");
    if (n > 0 && !D) fail(SRTC_ERR_ARG, "null D");
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    Ctx *c = &ctx->c;
    validate_operand(c, SRTC_MIN_PLUS, A, "A", s);  // O(nnz), small beside the n^2 path matrix
    Folded fa;
    fold_sparse(c, SRTC_MIN_PLUS, id, A, "ij", "i", "j", &fa, s);
    int32_t r = 0;
    apsp_tiskin(c, fa.view, (int32_t)id.i, D, H, &r, round_nnz, s);
    if (rounds_out) *rounds_out = r;
  });
}

int64_t srtc_mlp_num_params(void) {
  const int64_t K = SRTC_NUM_SCHEDULES;
  return 64 * 32 + 64 + 64 * 64 + 64 + K * 64 + K;
}

}  // extern "C"
