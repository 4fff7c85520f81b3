// Elementwise transforms and the Jacobi iteration (Section 4.1).
//
// Transforms (Section 3.4's user-defined transforms, here a fixed set of
// functor templates chosen by an enum): every element c of C is updated
// from the elements of A and B at the same letters; a letter of C missing
// from A or B broadcasts that operand along it (stride 0), which covers the
// listing's D["abij"] += Ei["i"] and the nested-loop example
// C["ij"] = C["ij"] / (A["i"] + B["j"]).
//
// Jacobi: x^{l+1}_i = (b_i - sum_{j != i} A_ij x^l_j) / A_ii until the
// residual b - A x is small.  One fused kernel per step forms the row sum
// once and gives both the update and the residual of the incoming iterate
// (r_i = b_i - sum_{j != i} A_ij x_j - A_ii x_i), so a step reads A once.
#include <algorithm>

#include "internal.hpp"

namespace srtc {

namespace {

struct BcastArgs {
  int64_t ext[SRTC_MAX_ORDER];  // C's extents
  int64_t sa[SRTC_MAX_ORDER];   // A's stride along C's mode q (0: broadcast)
  int64_t sb[SRTC_MAX_ORDER];
  int order;
  int64_t total;
};

template <class T, int OP>
__device__ __forceinline__ T apply(T a, T b, T c, T alpha) {
  if constexpr (OP == SRTC_TF_RECIP) return alpha / c;
  else if constexpr (OP == SRTC_TF_SCALE) return alpha * c;
  else if constexpr (OP == SRTC_TF_ADD) return c + alpha * a;
  else if constexpr (OP == SRTC_TF_FMA) return c + alpha * a * b;
  else return c / (a + b);  // SRTC_TF_DIV_SUM
}

template <class T, int OP>
__global__ void transform_dense(const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ C, BcastArgs g,
                                T alpha) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < g.total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e, oa = 0, ob = 0;
    for (int q = g.order - 1; q >= 0; q--) {
      const int64_t i = rem % g.ext[q];
      rem /= g.ext[q];
      oa += i * g.sa[q];
      ob += i * g.sb[q];
    }
    const T a = A ? A[oa] : (T)0, b = B ? B[ob] : (T)0;
    C[e] = apply<T, OP>(a, b, C[e], alpha);
  }
}

template <class T, int OP>
void launch_transform(const void *A, const void *B, void *C, const BcastArgs &g, double alpha, hipStream_t s) {
  const unsigned grid = (unsigned)std::min<int64_t>((g.total + 255) / 256, 65536);
  transform_dense<T, OP><<<grid, 256, 0, s>>>((const T *)A, (const T *)B, (T *)C, g, (T)alpha);
  SRTC_LAUNCH_CHECK("transform_dense");
}

template <class T>
void transform_typed(int op, const void *A, const void *B, void *C, const BcastArgs &g, double alpha, hipStream_t s) {
  switch (op) {
    case SRTC_TF_RECIP: launch_transform<T, SRTC_TF_RECIP>(A, B, C, g, alpha, s); break;
    case SRTC_TF_SCALE: launch_transform<T, SRTC_TF_SCALE>(A, B, C, g, alpha, s); break;
    case SRTC_TF_ADD: launch_transform<T, SRTC_TF_ADD>(A, B, C, g, alpha, s); break;
    case SRTC_TF_FMA: launch_transform<T, SRTC_TF_FMA>(A, B, C, g, alpha, s); break;
    case SRTC_TF_DIV_SUM: launch_transform<T, SRTC_TF_DIV_SUM>(A, B, C, g, alpha, s); break;
    default: fail(SRTC_ERR_ARG, "unknown transform");
  }
}

// ------------------------------------------------------------- Jacobi --

// The diagonal of each row (0 where missing); bad[0] set if any is 0.
template <class T>
__global__ void jacobi_diag(const int64_t *__restrict__ rp, const int32_t *__restrict__ col, const T *__restrict__ val,
                            int64_t n, T *__restrict__ d, int32_t *bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    T dii = 0;
    for (int64_t p = rp[i]; p < rp[i + 1]; p++)
      if (col[p] == i) dii += val[p];
    d[i] = dii;
    if (dii == (T)0) atomicOr(bad, 1);
  }
}

// One Jacobi step for G lanes per row: x_out = (b - R x_in) / d and the
// block's partial sum of r_i^2 for r = b - A x_in (fp64), written to
// part[blockIdx.x].  256 threads per block, a grid-stride loop over rows.
// Does nothing once the iteration has stopped (st->done), so the steps
// of a replayed graph after the stopping one leave both buffers alone.
template <class T, int G>
__global__ void __launch_bounds__(256) jacobi_step(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                   const T *__restrict__ val, const T *__restrict__ d,
                                                   const T *__restrict__ b, const T *__restrict__ x_in,
                                                   T *__restrict__ x_out, int64_t n, double *__restrict__ part,
                                                   const JacobiState *__restrict__ st) {
  __shared__ double red[256 / WAVE];
  if (st->done) return;  // uniform over the grid
  const int lane = lane_id(), sub = lane % G;
  const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / G;
  double rr = 0.0;
  // the G lanes of a row are one aligned lane group, so the shuffles below
  // stay inside lanes that take the same trips
  for (int64_t i = grp; i < n; i += ngrp) {
    // the row's own terms first, so their loads overlap the row sum
    const double bi = sub == 0 ? (double)b[i] : 0.0, di = sub == 0 ? (double)d[i] : 0.0;
    const double xi = sub == 0 ? (double)x_in[i] : 0.0;
    const int64_t p1 = rp[i + 1];
    double s = 0.0;
    // four entries per lane per pass, all loads issued before the sums;
    // padding uses column i, which the diagonal test skips
    for (int64_t p = rp[i] + sub; p < p1; p += 4 * G) {
      int32_t j[4];
      T v[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const bool ok = p + u * G < p1;
        j[u] = ok ? col[p + u * G] : (int32_t)i;
        v[u] = ok ? val[p + u * G] : (T)0;
      }
      double xv[4];
#pragma unroll
      for (int u = 0; u < 4; u++) xv[u] = j[u] != i ? (double)x_in[j[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; u++) s += (double)v[u] * xv[u];
    }
#pragma unroll
    for (int w = G / 2; w >= 1; w >>= 1) s += __shfl_xor(s, w, G);
    if (sub == 0) {
      x_out[i] = (T)((bi - s) / di);
      const double r = bi - s - di * xi;
      rr += r * r;
    }
  }
  rr = wave_sum(rr);
  if (lane == 0) red[threadIdx.x / WAVE] = rr;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 256 / WAVE; w++) t += red[w];
    part[blockIdx.x] = t;
  }
}

// The residual of the step's incoming iterate x^l (l = st->iter): the sum
// of part[0..nb) in a fixed order (one block of 256 threads).  Stops the
// iteration when l >= 1 and |r|^2 <= tol2, else moves on to x^{l+1}.
__global__ void __launch_bounds__(256) jacobi_reduce(const double *__restrict__ part, int64_t nb,
                                                     JacobiState *__restrict__ st, double tol2) {
  __shared__ double red[256 / WAVE];
  if (st->done) return;  // uniform over the block
  double t = 0.0;
  for (int64_t q = threadIdx.x; q < nb; q += 256) t += part[q];
  t = wave_sum(t);
  if (lane_id() == 0) red[threadIdx.x / WAVE] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double u = 0.0;
    for (int w = 0; w < 256 / WAVE; w++) u += red[w];
    st->rsq = u;
    if (st->iter >= 1 && u <= tol2) st->done = 1;
    else st->iter += 1;
  }
}

}  // namespace

void transform_dense_call(int op, int dt, double alpha, const int64_t *cext, int order, const void *A,
                          const int64_t *sa, const void *B, const int64_t *sb, void *C, hipStream_t s) {
  BcastArgs g{};
  g.order = order;
  g.total = 1;
  for (int q = 0; q < order; q++) {
    g.ext[q] = cext[q];
    g.sa[q] = sa[q];
    g.sb[q] = sb[q];
    g.total *= cext[q];
  }
  if (g.total == 0) return;
  if (dt == SRTC_F64) transform_typed<double>(op, A, B, C, g, alpha, s);
  else if (dt == SRTC_F32) transform_typed<float>(op, A, B, C, g, alpha, s);
  else fail(SRTC_ERR_DTYPE, "transforms are defined for F64 and F32");
}

void JacobiPlan::build(Ctx *c, int dt_, const CsrView &A_, hipStream_t s) {
  ctx = c;
  dt = dt_;
  A = A_;
  const int64_t n = A.m;
  const double avg = n > 0 ? (double)A.nnz / (double)n : 1.0;
  // about four nonzeros per lane: more rows in flight per wave hides the
  // dependent loads of a row (row pointer, then columns, then x)
  G = 4;
  while (G < 64 && 4 * G < avg) G <<= 1;
  grid = (int)std::max<int64_t>(1, std::min<int64_t>((n * G + 255) / 256, 16384));
  const size_t es = dtype_size(dt);
  dbuf = Buf(c, es * (size_t)std::max<int64_t>(n, 1));
  part = Buf(c, sizeof(double) * (size_t)grid);
  Buf bad(c, 64);
  fill_i32(bad.as<int32_t>(), 1, 0, s);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
  if (n > 0) {
    if (dt == SRTC_F64)
      jacobi_diag<double><<<g, 256, 0, s>>>(A.rowptr, A.col, (const double *)A.val, n, dbuf.as<double>(),
                                             bad.as<int32_t>());
    else
      jacobi_diag<float><<<g, 256, 0, s>>>(A.rowptr, A.col, (const float *)A.val, n, dbuf.as<float>(),
                                            bad.as<int32_t>());
    SRTC_LAUNCH_CHECK("jacobi_diag");
  }
  int32_t h = 0;
  read_to_host(c, &h, bad.p, sizeof(h), s);
  if (h) fail(SRTC_ERR_ARG, "Jacobi needs a nonzero diagonal entry in every row");
}

template <class T, int G>
static void step_typed(const JacobiPlan &pl, const void *b, const void *x_in, void *x_out, JacobiState *st,
                       double tol2, hipStream_t s) {
  jacobi_step<T, G><<<pl.grid, 256, 0, s>>>(pl.A.rowptr, pl.A.col, (const T *)pl.A.val, pl.dbuf.as<T>(),
                                            (const T *)b, (const T *)x_in, (T *)x_out, pl.A.m, pl.part.as<double>(),
                                            st);
  SRTC_LAUNCH_CHECK("jacobi_step");
  jacobi_reduce<<<1, 256, 0, s>>>(pl.part.as<double>(), pl.grid, st, tol2);
  SRTC_LAUNCH_CHECK("jacobi_reduce");
}

template <class T>
static void step_width(const JacobiPlan &pl, const void *b, const void *x_in, void *x_out, JacobiState *st,
                       double tol2, hipStream_t s) {
  switch (pl.G) {
    case 4: step_typed<T, 4>(pl, b, x_in, x_out, st, tol2, s); break;
    case 8: step_typed<T, 8>(pl, b, x_in, x_out, st, tol2, s); break;
    case 16: step_typed<T, 16>(pl, b, x_in, x_out, st, tol2, s); break;
    case 32: step_typed<T, 32>(pl, b, x_in, x_out, st, tol2, s); break;
    default: step_typed<T, 64>(pl, b, x_in, x_out, st, tol2, s); break;
  }
}

void jacobi_step_call(const JacobiPlan &pl, const void *b, const void *x_in, void *x_out, JacobiState *st,
                      double tol2, hipStream_t s) {
  ProfScope ps(pl.ctx, "jacobi.step",
               (4.0 + (double)dtype_size(pl.dt)) * (double)pl.A.nnz + 8.0 * (double)(pl.A.m + 1) +
                   4.0 * (double)dtype_size(pl.dt) * (double)pl.A.m,
               s);
  if (pl.dt == SRTC_F64) step_width<double>(pl, b, x_in, x_out, st, tol2, s);
  else step_width<float>(pl, b, x_in, x_out, st, tol2, s);
}

}  // namespace srtc
