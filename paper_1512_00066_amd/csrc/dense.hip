// Dense (+,x) tiles on the matrix cores, and dense mode permutation.
//
// Dense operands appear where a contraction has no sparsity to exploit; the
// paper's dense baseline runs such products as BLAS GEMM and notes that small
// dense blocks inside sparse data are worth exploiting (Section 6).  Only the
// (+,x) semiring maps onto MFMA; tropical, boolean and (max,x) products have
// no matrix-core form.
//
// Tile: 64x64 outputs per 256-thread block, each wave a 32x32 quadrant made
// of 2x2 MFMA 16x16 tiles; K is staged through LDS 16 at a time.
//   fp64: V_MFMA_F64_16X16X4_F64, fp64 accumulation.
//   fp32: V_MFMA_F32_16X16X4_F32, with the fp32 accumulators added into fp64
//         registers every 128 K-steps, so a dot product of any length keeps
//         the relative error of an fp32 sum of at most 128 terms.
#include <algorithm>

#include "internal.hpp"

namespace srtc {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 16;

// Batch z of a strided batch (grid z, grid-stride over batches) multiplies
// A + z M K by B + z K N into C + z M N.
template <class T>
__global__ void __launch_bounds__(256) gemm_mfma(const T *__restrict__ A0, const T *__restrict__ B0, T *__restrict__ C0,
                                                 int64_t M, int64_t N, int64_t K, int accumulate, int64_t batch) {
  __shared__ T As[TM][TK + 1];
  __shared__ T Bs[TK][TN + 1];
  for (int64_t z = blockIdx.z; z < batch; z += gridDim.z) {
    const T *__restrict__ A = A0 + z * M * K;
    const T *__restrict__ B = B0 + z * K * N;
    T *__restrict__ C = C0 + z * M * N;
    const int t = threadIdx.x;
    const int w = t / WAVE, l = lane_id();
    const int64_t m0 = (int64_t)blockIdx.y * TM, n0 = (int64_t)blockIdx.x * TN;
    const int wm = (w / 2) * 32, wn = (w % 2) * 32;  // wave quadrant
    double acc64[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++)
#pragma unroll
        for (int q = 0; q < 4; q++) acc64[a][b][q] = 0.0;
    v4f acc32[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++) acc32[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    v4d accd[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++) accd[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    int since_flush = 0;
    for (int64_t k0 = 0; k0 < K; k0 += TK) {
      // stage A (64x16) and B (16x64): 1024 elements each, 4 per thread
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int e = t + r * 256;
        const int am = e / TK, ak = e % TK;
        const int64_t gm = m0 + am, gk = k0 + ak;
        As[am][ak] = (gm < M && gk < K) ? A[gm * K + gk] : (T)0;
        const int bk = e / TN, bn = e % TN;
        const int64_t gk2 = k0 + bk, gn = n0 + bn;
        Bs[bk][bn] = (gk2 < K && gn < N) ? B[gk2 * N + gn] : (T)0;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < TK; kk += 4) {
        T av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; a++) av[a] = As[wm + a * 16 + (l % 16)][kk + l / 16];
#pragma unroll
        for (int b = 0; b < 2; b++) bv[b] = Bs[kk + l / 16][wn + b * 16 + (l % 16)];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
          for (int b = 0; b < 2; b++) {
            if constexpr (sizeof(T) == 8)
              accd[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], accd[a][b], 0, 0, 0);
            else
              acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc32[a][b], 0, 0, 0);
          }
      }
      __syncthreads();
      if constexpr (sizeof(T) == 4) {
        since_flush += TK;
        if (since_flush >= 128) {
#pragma unroll
          for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++) {
#pragma unroll
              for (int q = 0; q < 4; q++) acc64[a][b][q] += (double)acc32[a][b][q];
              acc32[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
            }
          since_flush = 0;
        }
      }
    }
    // output layout of a 16x16 MFMA tile, lane l, column l%16, accumulator q:
    //   fp32 (16x16x4 f32): row 4*(l/16) + q
    //   fp64 (16x16x4 f64): row 4*q + l/16
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int b = 0; b < 2; b++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
          double v;
          if constexpr (sizeof(T) == 8) v = accd[a][b][q];
          else v = acc64[a][b][q] + (double)acc32[a][b][q];
          const int64_t gm = m0 + wm + a * 16 + (sizeof(T) == 8 ? 4 * q + l / 16 : 4 * (l / 16) + q);
          const int64_t gn = n0 + wn + b * 16 + (l % 16);
          if (gm < M && gn < N) {
            if (accumulate) v += (double)C[gm * N + gn];
            C[gm * N + gn] = (T)v;
          }
        }
    __syncthreads();  // the next batch restages As and Bs
  }
}

// Large tiles: 128x128 outputs per 256-thread block, each wave a 64x64
// quadrant of 4x4 MFMA 16x16 tiles (16 MFMAs per 4-deep k step against 8
// fragment reads), the next 32-deep k-tile prefetched into registers while
// the current one is multiplied.  Used when both output sides reach 128.
constexpr int BM = 128, BN = 128, BK = 32;

template <class T>
__global__ void __launch_bounds__(256) gemm_mfma_128(const T *__restrict__ A0, const T *__restrict__ B0,
                                                     T *__restrict__ C0, int64_t M, int64_t N, int64_t K,
                                                     int accumulate, int64_t batch) {
  __shared__ T As[BM][BK + 1];
  __shared__ T Bs[BK][BN + 1];
  constexpr int LA = BM * BK / 256, LB = BK * BN / 256;  // staged elements per thread
  const int t = threadIdx.x;
  const int w = t / WAVE, l = lane_id();
  const int wm = (w / 2) * 64, wn = (w % 2) * 64;
  for (int64_t z = blockIdx.z; z < batch; z += gridDim.z) {
    const T *__restrict__ A = A0 + z * M * K;
    const T *__restrict__ B = B0 + z * K * N;
    T *__restrict__ C = C0 + z * M * N;
    const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
    v4d accd[4][4];
    v4f acc32[4][4];
    double acc64[4][4][4];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++) {
        if constexpr (sizeof(T) == 8) {
          accd[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
        } else {
          acc32[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < 4; q++) acc64[a][b][q] = 0.0;
        }
      }
    T ra[LA], rb[LB];
    auto fetch = [&](int64_t k0) {
#pragma unroll
      for (int r = 0; r < LA; r++) {
        const int e = t + r * 256, am = e / BK, ak = e % BK;
        const int64_t gm = m0 + am, gk = k0 + ak;
        ra[r] = (gm < M && gk < K) ? A[gm * K + gk] : (T)0;
      }
#pragma unroll
      for (int r = 0; r < LB; r++) {
        const int e = t + r * 256, bk = e / BN, bn = e % BN;
        const int64_t gk = k0 + bk, gn = n0 + bn;
        rb[r] = (gk < K && gn < N) ? B[gk * N + gn] : (T)0;
      }
    };
    fetch(0);
    int since_flush = 0;
    for (int64_t k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
      for (int r = 0; r < LA; r++) {
        const int e = t + r * 256;
        As[e / BK][e % BK] = ra[r];
      }
#pragma unroll
      for (int r = 0; r < LB; r++) {
        const int e = t + r * 256;
        Bs[e / BN][e % BN] = rb[r];
      }
      __syncthreads();
      if (k0 + BK < K) fetch(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        T av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; a++) av[a] = As[wm + a * 16 + (l % 16)][kk + l / 16];
#pragma unroll
        for (int b = 0; b < 4; b++) bv[b] = Bs[kk + l / 16][wn + b * 16 + (l % 16)];
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
          for (int b = 0; b < 4; b++) {
            if constexpr (sizeof(T) == 8)
              accd[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], accd[a][b], 0, 0, 0);
            else
              acc32[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc32[a][b], 0, 0, 0);
          }
      }
      __syncthreads();
      if constexpr (sizeof(T) == 4) {
        since_flush += BK;
        if (since_flush >= 128) {
#pragma unroll
          for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) {
#pragma unroll
              for (int q = 0; q < 4; q++) acc64[a][b][q] += (double)acc32[a][b][q];
              acc32[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
            }
          since_flush = 0;
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
          double v;
          if constexpr (sizeof(T) == 8) v = accd[a][b][q];
          else v = acc64[a][b][q] + (double)acc32[a][b][q];
          const int64_t gm = m0 + wm + a * 16 + (sizeof(T) == 8 ? 4 * q + l / 16 : 4 * (l / 16) + q);
          const int64_t gn = n0 + wn + b * 16 + (l % 16);
          if (gm < M && gn < N) {
            if (accumulate) v += (double)C[gm * N + gn];
            C[gm * N + gn] = (T)v;
          }
        }
  }
}

struct PermArgs {
  int64_t sdims[SRTC_MAX_ORDER];   // source extents
  int64_t sstride[SRTC_MAX_ORDER]; // source strides
  int64_t odims[SRTC_MAX_ORDER];   // output extents (source mode perm[q])
  int perm[SRTC_MAX_ORDER];
  int order;
  int64_t total;
};

template <class E>
__global__ void permute_kernel(const E *__restrict__ src, E *__restrict__ dst, PermArgs a) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < a.total;
       o += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = o, si = 0;
    for (int q = a.order - 1; q >= 0; q--) {
      const int64_t idx = rem % a.odims[q];
      rem /= a.odims[q];
      si += idx * a.sstride[a.perm[q]];
    }
    dst[o] = src[si];
  }
}

// dst (in its own mode order) = src permuted, combined with dst's previous
// value by the semiring's (+); entries equal to the identity are absent.
template <class SR>
__global__ void permute_combine_kernel(const typename SR::val_t *__restrict__ src, typename SR::val_t *__restrict__ dst,
                                       PermArgs a, typename SR::acc_t id) {
  using A = typename SR::acc_t;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < a.total;
       o += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = o, si = 0;
    for (int q = a.order - 1; q >= 0; q--) {
      const int64_t idx = rem % a.odims[q];
      rem /= a.odims[q];
      si += idx * a.sstride[a.perm[q]];
    }
    A acc = id;
    const auto x = src[si], y = dst[o];
    if (!SR::absent(x, id)) acc = SR::add(acc, (A)x);
    if (!SR::absent(y, id)) acc = SR::add(acc, (A)y);
    dst[o] = out_clamped<SR>(acc, id);
  }
}

PermArgs perm_args(int order, const int64_t *dims, const int *perm) {
  PermArgs a{};
  a.order = order;
  a.total = 1;
  int64_t st = 1;
  for (int q = order - 1; q >= 0; q--) {
    a.sdims[q] = dims[q];
    a.sstride[q] = st;
    st *= dims[q];
  }
  for (int q = 0; q < order; q++) {
    a.perm[q] = perm[q];
    a.odims[q] = dims[perm[q]];
    a.total *= dims[q];
  }
  return a;
}

struct CombineCall {
  IdVal id;
  const void *src;
  void *dst;
  PermArgs a;
  hipStream_t s;
};

template <class SR> void permute_combine_typed(const CombineCall &q) {
  using V = typename SR::val_t;
  const unsigned grid = (unsigned)std::min<int64_t>((q.a.total + 255) / 256, 65536);
  permute_combine_kernel<SR><<<grid, 256, 0, q.s>>>((const V *)q.src, (V *)q.dst, q.a, id_as<SR>(q.id));
  SRTC_LAUNCH_CHECK("permute_combine_kernel");
}

// C = A (x) B elementwise, combined with C's previous value by (+) when
// accumulating; identity operands give the identity.
template <class SR>
__global__ void hadamard_kernel(const typename SR::val_t *__restrict__ A, const typename SR::val_t *__restrict__ B,
                                typename SR::val_t *__restrict__ C, int64_t n, int accumulate,
                                typename SR::acc_t id) {
  using Acc = typename SR::acc_t;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const auto a = A[e], b = B[e];
    Acc acc = id;
    if (!SR::absent(a, id) && !SR::absent(b, id)) acc = SR::mul(a, b);
    if (accumulate) {
      const auto y = C[e];
      if (!SR::absent(y, id)) acc = SR::add(acc, (Acc)y);
    }
    C[e] = out_clamped<SR>(acc, id);
  }
}

struct HadamardCall {
  IdVal id;
  const void *A, *B;
  void *C;
  int64_t n;
  int accumulate;
  hipStream_t s;
};

template <class SR> void hadamard_typed(const HadamardCall &q) {
  using V = typename SR::val_t;
  const unsigned grid = (unsigned)std::min<int64_t>((q.n + 255) / 256, 65536);
  hadamard_kernel<SR><<<grid, 256, 0, q.s>>>((const V *)q.A, (const V *)q.B, (V *)q.C, q.n, q.accumulate,
                                             id_as<SR>(q.id));
  SRTC_LAUNCH_CHECK("hadamard_kernel");
}

}  // namespace

void dense_hadamard(int sr, int dt, IdVal id, const void *A, const void *B, void *C, int64_t n, int accumulate,
                    hipStream_t s) {
  if (n <= 0) return;
  HadamardCall q{id, A, B, C, n, accumulate, s};
  SRTC_DISPATCH_SR(sr, dt, hadamard_typed, q);
}

void dense_permute_combine(int sr, int dt, IdVal id, const void *src, void *dst, int order, const int64_t *dims,
                           const int *perm, hipStream_t s) {
  CombineCall q{id, src, dst, perm_args(order, dims, perm), s};
  if (q.a.total == 0) return;
  SRTC_DISPATCH_SR(sr, dt, permute_combine_typed, q);
}

void dense_gemm_plus_times(Ctx *, int dt, const void *A, const void *B, void *C, int64_t M, int64_t N, int64_t K,
                           int accumulate, hipStream_t s, int64_t batch) {
  if (M == 0 || N == 0 || batch <= 0) return;
  if (M >= BM && N >= BN) {
    dim3 g((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)std::min<int64_t>(batch, 65535));
    if (g.y > 65535) fail(SRTC_ERR_UNSUPPORTED, "dense gemm: too many row tiles");
    if (dt == SRTC_F64)
      gemm_mfma_128<double><<<g, 256, 0, s>>>((const double *)A, (const double *)B, (double *)C, M, N, K, accumulate,
                                               batch);
    else if (dt == SRTC_F32)
      gemm_mfma_128<float><<<g, 256, 0, s>>>((const float *)A, (const float *)B, (float *)C, M, N, K, accumulate,
                                              batch);
    else
      fail(SRTC_ERR_DTYPE, "dense (+,x) needs F64 or F32");
    SRTC_LAUNCH_CHECK("gemm_mfma_128");
    return;
  }
  dim3 grid((unsigned)((N + TN - 1) / TN), (unsigned)((M + TM - 1) / TM),
            (unsigned)std::min<int64_t>(batch, 65535));
  if (grid.y > 65535) fail(SRTC_ERR_UNSUPPORTED, "dense gemm: too many row tiles");
  if (dt == SRTC_F64)
    gemm_mfma<double><<<grid, 256, 0, s>>>((const double *)A, (const double *)B, (double *)C, M, N, K, accumulate,
                                            batch);
  else if (dt == SRTC_F32)
    gemm_mfma<float><<<grid, 256, 0, s>>>((const float *)A, (const float *)B, (float *)C, M, N, K, accumulate,
                                           batch);
  else
    fail(SRTC_ERR_DTYPE, "dense (+,x) needs F64 or F32");
  SRTC_LAUNCH_CHECK("gemm_mfma");
}

void dense_permute(const void *src, void *dst, int esize, int order, const int64_t *dims, const int *perm,
                   hipStream_t s) {
  const PermArgs a = perm_args(order, dims, perm);
  if (a.total == 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>((a.total + 255) / 256, 65536);
  switch (esize) {
    case 8: permute_kernel<uint64_t><<<grid, 256, 0, s>>>((const uint64_t *)src, (uint64_t *)dst, a); break;
    case 4: permute_kernel<uint32_t><<<grid, 256, 0, s>>>((const uint32_t *)src, (uint32_t *)dst, a); break;
    default: permute_kernel<uint8_t><<<grid, 256, 0, s>>>((const uint8_t *)src, (uint8_t *)dst, a); break;
  }
  SRTC_LAUNCH_CHECK("permute_kernel");
}

}  // namespace srtc
