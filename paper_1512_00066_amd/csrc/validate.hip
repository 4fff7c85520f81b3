// Operand structure checks (requested with srtc_opts.validate).
//
// A CSR operand must have rowptr[0] = 0, non-decreasing row pointers ending
// at nnz, columns in [0, ncols) and strictly ascending within each row (the
// canonical form the fold produces; the dense accumulator windows rely on
// the order).  COO keys must lie in [0, product of dims).  Float (min,+)
// values may not be NaN or -inf (the identity +inf is allowed); int32
// (min,+) values must lie in [-id, id].  Every read
// stays inside the operand's declared extents, so a malformed operand is
// reported, never dereferenced out of range.
#include <cmath>

#include "internal.hpp"

namespace srtc {

namespace {

enum : int32_t {
  BAD_ROWPTR_START = 1,
  BAD_ROWPTR_ORDER = 2,
  BAD_ROWPTR_END = 4,
  BAD_COL_RANGE = 8,
  BAD_COL_ORDER = 16,
  BAD_KEY_RANGE = 32,
  BAD_VALUE = 64,
  BAD_RANGE = 128,
};

__global__ void check_csr_kernel(const int64_t *__restrict__ rp, int64_t m, const int32_t *__restrict__ col,
                                 int64_t nnz, int64_t ncols, int32_t *err) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  const int lane = lane_id();
  int32_t bad = 0;
  for (int64_t i = wid; i < m; i += nw) {
    const int64_t a = rp[i], b = rp[i + 1];
    if (i == 0 && a != 0) bad |= BAD_ROWPTR_START;
    if (i == m - 1 && b != nnz) bad |= BAD_ROWPTR_END;
    if (b < a) bad |= BAD_ROWPTR_ORDER;
    const int64_t lo = max((int64_t)0, min(a, nnz)), hi = max((int64_t)0, min(b, nnz));
    for (int64_t p = lo + lane; p < hi; p += WAVE) {
      const int32_t c = col[p];
      if (c < 0 || c >= ncols) bad |= BAD_COL_RANGE;
      if (p + 1 < hi && col[p + 1] <= c) bad |= BAD_COL_ORDER;
    }
  }
  if (bad) atomicOr(err, bad);
}

__global__ void check_keys_kernel(const int64_t *__restrict__ keys, int64_t nnz, int64_t total, int32_t *err) {
  int32_t bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = keys[e];
    if (k < 0 || k >= total) bad |= BAD_KEY_RANGE;
  }
  if (bad) atomicOr(err, bad);
}

template <class T>
__global__ void check_tropical_kernel(const T *__restrict__ v, int64_t n, int32_t *err) {
  int32_t bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const T x = v[e];
    if (x != x || (x < (T)0 && isinf(x))) bad |= BAD_VALUE;
  }
  if (bad) atomicOr(err, bad);
}

// (min,+) int32 operands must lie in [-id, id] so that no sum of two
// overflows int32 (the identity is at most INT32_MAX / 2).
__global__ void check_tropical_i32_kernel(const int32_t *__restrict__ v, int64_t n, int32_t id, int32_t *err) {
  int32_t bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = v[e];
    if (x < -id || x > id) bad |= BAD_RANGE;
  }
  if (bad) atomicOr(err, bad);
}

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

}  // namespace

void validate_operand(Ctx *c, int sr, const srtc_tensor *t, const char *name, hipStream_t s, const IdVal *id) {
  if (t->format == SRTC_DENSE) return;
  Buf err(c, 64);
  fill_i32(err.as<int32_t>(), 1, 0, s);
  int64_t nvals = t->nnz;
  if (t->format == SRTC_CSR) {
    int64_t m = 1, n = 1;
    for (int i = 0; i < t->split; i++) m *= t->dims[i];
    for (int i = t->split; i < t->order; i++) n *= t->dims[i];
    if (m > 0) {
      check_csr_kernel<<<grid_of(m * WAVE), 256, 0, s>>>(t->rowptr, m, t->colidx, t->nnz, n, err.as<int32_t>());
      SRTC_LAUNCH_CHECK("check_csr_kernel");
    }
  } else if (t->nnz > 0) {
    int64_t total = 1;
    for (int i = 0; i < t->order; i++) total *= t->dims[i];
    check_keys_kernel<<<grid_of(t->nnz), 256, 0, s>>>(t->coo_keys, t->nnz, total, err.as<int32_t>());
    SRTC_LAUNCH_CHECK("check_keys_kernel");
  }
  if (sr == SRTC_MIN_PLUS && nvals > 0) {
    if (t->dtype == SRTC_F32)
      check_tropical_kernel<float><<<grid_of(nvals), 256, 0, s>>>((const float *)t->vals, nvals, err.as<int32_t>());
    if (t->dtype == SRTC_I32 && id)
      check_tropical_i32_kernel<<<grid_of(nvals), 256, 0, s>>>((const int32_t *)t->vals, nvals, (int32_t)id->i,
                                                               err.as<int32_t>());
    SRTC_LAUNCH_CHECK("check_tropical_kernel");
  }
  int32_t bad = 0;
  read_to_host(c, &bad, err.p, sizeof(bad), s);
  if (!bad) return;
  std::string msg = std::string(name) + ":";
  if (bad & BAD_ROWPTR_START) msg += " rowptr[0] != 0;";
  if (bad & BAD_ROWPTR_ORDER) msg += " rowptr decreases;";
  if (bad & BAD_ROWPTR_END) msg += " rowptr[m] != nnz;";
  if (bad & BAD_COL_RANGE) msg += " column index out of range;";
  if (bad & BAD_COL_ORDER) msg += " columns not strictly ascending within a row;";
  if (bad & BAD_KEY_RANGE) msg += " COO key out of range;";
  if (bad & BAD_VALUE) msg += " NaN or -inf value for (min,+);";
  if (bad & BAD_RANGE) msg += " (min,+) int32 value outside [-identity, identity];";
  fail(SRTC_ERR_FORMAT, msg);
}

}  // namespace srtc
