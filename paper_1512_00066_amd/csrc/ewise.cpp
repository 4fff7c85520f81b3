// Element-wise (+) of two sparse matrices of the same shape: the union of
// the patterns, with entries present in both combined (X's value first).
// This is the "+=" of an indexed summation (Section 3.3.1), used when a
// sparse contraction accumulates into an existing output.
#include "internal.hpp"

namespace srtc {

void ewise_add(Ctx *c, int sr, int dt, IdVal id, const CsrView &X, const CsrView &Y, CsrOut *out, hipStream_t s) {
  if (X.m != Y.m || X.n != Y.n) fail(SRTC_ERR_DIM, "ewise_add: shapes differ");
  const int64_t nnz = X.nnz + Y.nnz;
  const size_t es = dtype_size(dt);
  Buf keys(c, sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
  Buf vals(c, es * (size_t)(nnz > 0 ? nnz : 1));
  csr_to_keys(X, keys.as<int64_t>(), s);
  csr_to_keys(Y, keys.as<int64_t>() + X.nnz, s);
  if (X.nnz) SRTC_HIP(hipMemcpyAsync(vals.p, X.val, es * (size_t)X.nnz, hipMemcpyDeviceToDevice, s));
  if (Y.nnz)
    SRTC_HIP(hipMemcpyAsync((char *)vals.p + es * (size_t)X.nnz, Y.val, es * (size_t)Y.nnz, hipMemcpyDeviceToDevice, s));
  fold_keys_to_csr(c, sr, dt, id, keys.as<int64_t>(), vals.p, nnz, X.m, X.n, out, s);
}

}  // namespace srtc
