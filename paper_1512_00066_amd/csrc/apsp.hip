// All-pairs shortest paths by Tiskin's path doubling (Section 4.2).
//
// P holds, for every pair, the lightest path found so far as a packed
// (weight, hops) value over the hop-carrying (min,+) semiring (ties go to
// fewer hops).  Round l (l = 1, 2, 4, ...) keeps in a sparse Pl only the
// entries of P whose path has exactly l hops and updates
//   P <- P (+) Pl (x) P.
// Every shortest path of at most 2l hops either has at most l hops or
// splits into a shortest path of exactly l hops followed by one of at most
// l hops, so after the round P covers all shortest paths of up to 2l hops;
// the listing's loop runs while l < n.  With the fewest-hops tie rule the
// l-hop prefix of a fewest-hops shortest path is itself a fewest-hops
// shortest path, so it is in Pl.  When Pl is empty no path has more than l
// hops and the loop stops early.
//
// Layout: P is dense n x n row-major uint64 (weight << 32 | hops); Pl is a
// CSR built from P each round; the product is the library's semiring SpMM
// with Pl as the sparse operand, the full n-wide P as the dense one, and
// the old P accumulated into the result (out of place: both factors are
// read before P changes).
#include <algorithm>
#include <utility>

#include "internal.hpp"

namespace srtc {

namespace {

unsigned grid_of(int64_t n, int bs = 256) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + bs - 1) / bs, 65536));
}

__global__ void apsp_init(uint64_t *__restrict__ P, int64_t n, uint64_t idv) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    P[e] = (e / n == e % n) ? 0ull : idv;  // zero-hop paths on the diagonal
}

// A wave per row; repeated entries of a row meet in a 64-bit atomic min.
__global__ void apsp_edges(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const int32_t *__restrict__ w, int64_t n, int32_t idw, uint64_t *__restrict__ P,
                           int32_t *bad) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t i = wid; i < n; i += nw) {
    for (int64_t p = rp[i] + lane_id(); p < rp[i + 1]; p += WAVE) {
      const int32_t x = w[p];
      if (x < 0) {
        atomicOr(bad, 1);
        continue;
      }
      if (x >= idw) continue;
      const uint64_t v = ((uint64_t)(uint32_t)x << 32) | 1ull;
      atomicMin((unsigned long long *)(P + i * n + col[p]), (unsigned long long)v);
    }
  }
}

// Largest weight and hop count over the 256 threads of a block, written
// to part[2 * blk] and part[2 * blk + 1] by thread 0 (all threads call it).
__device__ __forceinline__ void block_range(uint32_t wmax, uint32_t hmax, uint32_t *part, int64_t blk) {
  __shared__ uint32_t sw[4], sh[4];
  for (int d = WAVE / 2; d >= 1; d >>= 1) {
    const uint32_t ow = __shfl_xor(wmax, d, WAVE), oh = __shfl_xor(hmax, d, WAVE);
    wmax = ow > wmax ? ow : wmax;
    hmax = oh > hmax ? oh : hmax;
  }
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    sw[w] = wmax;
    sh[w] = hmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = sw[0], b = sh[0];
    for (int k = 1; k < 4; k++) {
      a = sw[k] > a ? sw[k] : a;
      b = sh[k] > b ? sh[k] : b;
    }
    part[2 * blk] = a;
    part[2 * blk + 1] = b;
  }
}

// Entries of row i whose path has exactly l hops (wave per row), and per
// block the largest weight and hop count of any path in P, which bound the
// values a round can form.  256 threads per block.
__global__ void __launch_bounds__(256) hops_count(const uint64_t *__restrict__ P, int64_t n, uint32_t l, uint32_t idw,
                                                  int64_t *__restrict__ cnt, uint32_t *__restrict__ part) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  uint32_t wmax = 0, hmax = 0;
  for (int64_t i = wid; i < n; i += nw) {
    int64_t c = 0;
#pragma unroll 8
    for (int64_t j = lane_id(); j < n; j += WAVE) {
      const uint64_t v = P[i * n + j];
      const uint32_t w = (uint32_t)(v >> 32), h = (uint32_t)v;
      const bool present = w < idw;
      c += (present && h == l) ? 1 : 0;
      if (present) {
        wmax = w > wmax ? w : wmax;
        hmax = h > hmax ? h : hmax;
      }
    }
    c = wave_sum(c);
    if (lane_id() == 0) cnt[i] = c;
  }
  block_range(wmax, hmax, part, blockIdx.x);
}

// info[0] = largest weight | largest hops << 32 over nb block partials,
// info[1] = *total (the count of l-hop paths).  One block of 256 threads.
__global__ void __launch_bounds__(256) range_reduce(const uint32_t *__restrict__ part, int64_t nb,
                                                    const int64_t *__restrict__ total, int64_t *__restrict__ info) {
  uint32_t wmax = 0, hmax = 0;
  for (int64_t b = threadIdx.x; b < nb; b += 256) {
    wmax = part[2 * b] > wmax ? part[2 * b] : wmax;
    hmax = part[2 * b + 1] > hmax ? part[2 * b + 1] : hmax;
  }
  uint32_t *res = reinterpret_cast<uint32_t *>(info);
  block_range(wmax, hmax, res, 0);
  if (threadIdx.x == 0) info[1] = *total;
}

__global__ void hops_fill(const uint64_t *__restrict__ P, int64_t n, uint32_t l, uint32_t idw,
                          const int64_t *__restrict__ rp, int32_t *__restrict__ col, uint64_t *__restrict__ val) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  const uint64_t lt = lanemask_lt();
  for (int64_t i = wid; i < n; i += nw) {
    int64_t pos = rp[i];
    for (int64_t j0 = 0; j0 < n; j0 += WAVE) {
      const int64_t j = j0 + lane_id();
      const uint64_t v = j < n ? P[i * n + j] : 0ull;
      const bool keep = j < n && (uint32_t)v == l && (uint32_t)(v >> 32) < idw;
      const uint64_t mk = __ballot(keep);
      if (keep) {
        const int64_t o = pos + __popcll(mk & lt);
        col[o] = (int32_t)j;
        val[o] = v;
      }
      pos += __popcll(mk);
    }
  }
}

// One round on dense tiles, for rounds whose sparse factor is dense enough:
//   Pn[i, j] = P[i, j] (+) (+)_k L[i, k] (x) P[k, j]
// with L[i, k] = P[i, k] where that path has exactly l hops, the identity
// elsewhere (masked while the tile is staged, so P_l is never built).  A
// block owns a TM x TN tile of Pn; 256 threads as 16 x 16, each holding
// RM x RN accumulators at rows ty RM + m and columns tx RN + q, so the LDS
// reads of a k step are one vector read each: a broadcast (L) and 16
// consecutive lanes' vectors (P).  The
// next k-tile is fetched into registers while the current one is used.
// An identity operand needs no test: its weight alone reaches the identity,
// which no accumulator exceeds (they start from P), so min() ignores it.
// k-tiles whose L part holds no l-hop entry are skipped.
//
// Values in the tiles (Enc):
//   Wide:   the packed path itself (64-bit add and compare per sum).
//   Narrow: (weight << hb) | hops in 32 bits with the identity 2^30, usable
//           when every path of the round fits: with W the largest weight
//           and H the largest hop count in P, sums have weight <= 2W and
//           hops <= l + H < 2^hb, and (2W + 1) << hb <= 2^30.  The map keeps
//           the order of paths and turns the path sum into one 32-bit add
//           (no carry out of the hop field) and the choice into one min.
struct Wide {
  using T = uint64_t;
  uint64_t idv;
  __device__ T enc(uint64_t x) const { return x; }
  __device__ T id() const { return idv; }
  __device__ uint64_t dec(T v) const { return v; }
};
struct Narrow {
  using T = uint32_t;
  uint32_t idw;
  int hb;
  __device__ T enc(uint64_t x) const {
    const uint32_t w = (uint32_t)(x >> 32);
    return w < idw ? ((w << hb) | (uint32_t)x) : (1u << 30);
  }
  __device__ T id() const { return 1u << 30; }
  // a sum may reach the identity weight when that is below 2^30 >> hb:
  // it is no path, as in the 64-bit form
  __device__ uint64_t dec(T v) const {
    return (v >= (1u << 30) || (v >> hb) >= idw)
               ? ((uint64_t)idw << 32)
               : (((uint64_t)(v >> hb) << 32) | (uint64_t)(v & ((1u << hb) - 1)));
  }
};

//
// With cnt given, the epilogue also counts for the next round (l2 = 2l):
// cnt[i] += entries of row i of Pn with exactly l2 hops (cnt zeroed by the
// caller), and part[2 b], part[2 b + 1] = largest weight and hop count in
// block b's tile, so the next round needs no separate pass over P.
template <class E, int TM, int TN, int TK, int MINB>
__global__ void __launch_bounds__(256, MINB) apsp_dense_round(const uint64_t *__restrict__ P, uint64_t *__restrict__ Pn,
                                                              int64_t n, uint32_t l, uint32_t idw, E enc,
                                                              int64_t *__restrict__ cnt, uint32_t l2,
                                                              uint32_t *__restrict__ part) {
  using T = typename E::T;
  constexpr int RM = TM / 16, RN = TN / 16;
  constexpr int LA = TM * TK / 256, LB = TK * TN / 256;  // staged words per thread
  static_assert(LA * 256 == TM * TK && LB * 256 == TK * TN, "tile must split over 256 threads");
  static_assert(256 % TK == 0 && 256 % TN == 0, "a thread keeps one column of each staged tile");
  // rows padded by 16 bytes: staging writes spread over banks and every
  // thread's RM rows (RN columns) stay one aligned 16-byte-multiple read
  __shared__ __align__(16) T Ls[TK][TM + 16 / sizeof(T)];
  __shared__ __align__(16) T Bs[TK][TN];
  const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
  const int64_t row0 = (int64_t)blockIdx.y * TM, col0 = (int64_t)blockIdx.x * TN;
  T acc[RM][RN];
#pragma unroll
  for (int m = 0; m < RM; m++)
#pragma unroll
    for (int q = 0; q < RN; q++) {
      const int64_t i = row0 + ty * RM + m, j = col0 + tx * RN + q;
      acc[m][q] = (i < n && j < n) ? enc.enc(P[i * n + j]) : enc.id();
    }
  // raw words of the next k-tile (identity pattern where out of range).
  // Thread tid stages column tid % TK of the L tile (rows tid / TK + t *
  // 256 / TK) and column tid % TN of the P tile (rows tid / TN + t * 256 /
  // TN), so each staged word is one running pointer plus a fixed stride.
  uint64_t ra[LA], rb[LB];
  const uint64_t idv = (uint64_t)idw << 32;
  const int ca = tid % TK, ra0 = tid / TK, cb = tid % TN, rb0 = tid / TN;
  const bool rows_in = row0 + TM <= n, cols_in = col0 + TN <= n;
  auto fetch = [&](int64_t k0) {
    const uint64_t *pa = P + (row0 + ra0) * n + k0 + ca;
    const uint64_t *pb = P + (k0 + rb0) * n + col0 + cb;
    const int64_t sa = (int64_t)(256 / TK) * n, sb = (int64_t)(256 / TN) * n;
    if (rows_in && cols_in && k0 + TK <= n) {
#pragma unroll
      for (int t = 0; t < LA; t++) ra[t] = pa[t * sa];
#pragma unroll
      for (int t = 0; t < LB; t++) rb[t] = pb[t * sb];
    } else {
#pragma unroll
      for (int t = 0; t < LA; t++)
        ra[t] = (row0 + ra0 + t * (256 / TK) < n && k0 + ca < n) ? pa[t * sa] : idv;
#pragma unroll
      for (int t = 0; t < LB; t++)
        rb[t] = (k0 + rb0 + t * (256 / TN) < n && col0 + cb < n) ? pb[t * sb] : idv;
    }
  };
  fetch(0);
  for (int64_t k0 = 0; k0 < n; k0 += TK) {
    int any = 0;
#pragma unroll
    for (int t = 0; t < LA; t++) {
      const uint64_t x = ra[t];
      const bool keep = (uint32_t)x == l && (uint32_t)(x >> 32) < idw;
      any |= keep ? 1 : 0;
      Ls[ca][ra0 + t * (256 / TK)] = keep ? enc.enc(x) : enc.id();
    }
#pragma unroll
    for (int t = 0; t < LB; t++) Bs[rb0 + t * (256 / TN)][cb] = enc.enc(rb[t]);
    const int live = __syncthreads_or(any);
    if (k0 + TK < n) fetch(k0 + TK);
    if (live) {
#pragma unroll 4
      for (int kk = 0; kk < TK; kk++) {
        T a[RM], b[RN];
#pragma unroll
        for (int m = 0; m < RM; m++) a[m] = Ls[kk][ty * RM + m];
#pragma unroll
        for (int q = 0; q < RN; q++) b[q] = Bs[kk][tx * RN + q];
#pragma unroll
        for (int m = 0; m < RM; m++)
#pragma unroll
          for (int q = 0; q < RN; q++) {
            const T c = a[m] + b[q];
            acc[m][q] = c < acc[m][q] ? c : acc[m][q];
          }
      }
    }
    __syncthreads();
  }
  uint32_t wmax = 0, hmax = 0;
#pragma unroll
  for (int m = 0; m < RM; m++) {
    const int64_t i = row0 + ty * RM + m;
    int c = 0;
#pragma unroll
    for (int q = 0; q < RN; q++) {
      const int64_t j = col0 + tx * RN + q;
      if (i < n && j < n) {
        const uint64_t o = enc.dec(acc[m][q]);
        Pn[i * n + j] = o;
        const uint32_t w = (uint32_t)(o >> 32), h = (uint32_t)o;
        if (w < idw) {
          c += h == l2 ? 1 : 0;
          wmax = w > wmax ? w : wmax;
          hmax = h > hmax ? h : hmax;
        }
      }
    }
    if (cnt) {
      // the 16 threads of a tile row are 16 consecutive lanes
      for (int d = 8; d >= 1; d >>= 1) c += __shfl_xor(c, d, WAVE);
      if (tx == 0 && i < n && c > 0) atomicAdd((unsigned long long *)(cnt + i), (unsigned long long)c);
    }
  }
  if (cnt) block_range(wmax, hmax, part, (int64_t)blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ void apsp_out(const uint64_t *__restrict__ P, int64_t total, uint32_t idw, int32_t *__restrict__ D,
                         int32_t *__restrict__ H) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t v = P[e];
    const uint32_t w = (uint32_t)(v >> 32);
    const bool reach = w < idw;
    D[e] = reach ? (int32_t)w : (int32_t)idw;
    if (H) H[e] = reach ? (int32_t)(uint32_t)v : -1;
  }
}

}  // namespace

// Declared in internal.hpp (used by the C entry point in capi.cpp).
// Rounds whose sparse factor holds at least this fraction of the n^2
// entries run on dense tiles; sparser ones as a CSR x dense product.  The
// crossover follows the measured rates: a 32-bit dense round forms its n^3
// sums about 18x faster per sum than the CSR product forms nnz * n, a
// 64-bit round about 7x.
constexpr double kDenseFracNarrow = 0.05, kDenseFracWide = 0.14;

void apsp_tiskin(Ctx *c, const CsrView &A, int32_t idw, int32_t *D, int32_t *H, int32_t *rounds, int64_t *round_nnz,
                 hipStream_t s) {
  const int64_t n = A.m;
  if (A.n != n) fail(SRTC_ERR_DIM, "apsp: A must be square");
  if (n > 0xffffffffll / 2) fail(SRTC_ERR_UNSUPPORTED, "apsp: too many vertices");
  if ((uint64_t)n * (uint64_t)n > (1ull << 40)) fail(SRTC_ERR_UNSUPPORTED, "apsp: dense n x n path matrix too large");
  const uint64_t idv = (uint64_t)(uint32_t)idw << 32;
  const int64_t total = n * n;
  Buf pa(c, sizeof(uint64_t) * (size_t)std::max<int64_t>(total, 1)), pb(c, sizeof(uint64_t) * (size_t)std::max<int64_t>(total, 1));
  // info[0] = value range, info[1] = count of l-hop paths (both per round),
  // info[2] = negative-weight flag (read with the first round's info)
  Buf info_b(c, 64);
  fill_i32(info_b.as<int32_t>(), 16, 0, s);
  int32_t *bad = reinterpret_cast<int32_t *>(info_b.as<int64_t>() + 2);
  uint64_t *P = pa.as<uint64_t>(), *Pn = pb.as<uint64_t>();
  {
    ProfScope ps(c, "apsp.init", 8.0 * (double)total, s);
    apsp_init<<<grid_of(total), 256, 0, s>>>(P, n, idv);
  }
  SRTC_LAUNCH_CHECK("apsp_init");
  if (A.nnz > 0) {
    ProfScope ps(c, "apsp.edges", 12.0 * (double)A.nnz + 8.0 * (double)(n + 1), s);
    apsp_edges<<<grid_of(n * WAVE), 256, 0, s>>>(A.rowptr, A.col, (const int32_t *)A.val, n, idw, P, bad);
    SRTC_LAUNCH_CHECK("apsp_edges");
  }
  if (n < 2) {
    // no round runs: check the weights here
    int32_t neg = 0;
    read_to_host(c, &neg, bad, sizeof(neg), s);
    if (neg) fail(SRTC_ERR_ARG, "apsp: negative edge weight");
  }
  const IdVal id{0.0, (int64_t)idw};
  Buf cnt(c, sizeof(int64_t) * (size_t)std::max<int64_t>(n, 1)), rp(c, sizeof(int64_t) * (size_t)(n + 1));
  // per-block ranges (hops_count's grid or a dense round's tiles) and the
  // reduced {range, count} the host reads once per round
  constexpr int DTM = 64, DTN = 64, DTK = 32;
  const int64_t cnt_blocks = std::min<int64_t>(grid_of(n * WAVE), 1024);
  const int64_t tiles = ((n + DTM - 1) / DTM) * ((n + DTN - 1) / DTN);
  Buf part(c, 8 * (size_t)std::max<int64_t>({cnt_blocks, tiles, 1}));
  bool counted = false;  // the previous dense round already counted this round's paths
  int32_t r = 0;
  if (round_nnz) std::fill(round_nnz, round_nnz + 64, (int64_t)0);
  for (int64_t l = 1; l < n; l <<= 1) {
    int64_t nparts = tiles;
    if (!counted) {
      nparts = cnt_blocks;
      ProfScope ps(c, "apsp.hops_count", 8.0 * (double)total + 8.0 * (double)n, s);
      hops_count<<<(unsigned)cnt_blocks, 256, 0, s>>>(P, n, (uint32_t)l, (uint32_t)idw, cnt.as<int64_t>(),
                                                      part.as<uint32_t>());
      SRTC_LAUNCH_CHECK("hops_count");
    }
    excl_scan_i64(c, cnt.as<int64_t>(), rp.as<int64_t>(), n, s);
    // one read per round: the value range and the count of l-hop paths
    range_reduce<<<1, 256, 0, s>>>(part.as<uint32_t>(), nparts, rp.as<int64_t>() + n, info_b.as<int64_t>());
    SRTC_LAUNCH_CHECK("range_reduce");
    int64_t info[3];
    read_to_host(c, info, info_b.p, sizeof(info), s);
    if (r == 0 && (int32_t)info[2]) fail(SRTC_ERR_ARG, "apsp: negative edge weight");
    const int64_t nnz = info[1];
    const uint32_t wmax = (uint32_t)info[0], hmax = (uint32_t)((uint64_t)info[0] >> 32);
    c->tracef("apsp: round %d, %lld paths of %lld hops", r, (long long)nnz, (long long)l);
    if (round_nnz && r < 64) round_nnz[r] = nnz;
    if (nnz == 0) break;  // no path has more than l hops
    const uint64_t hsum = (uint64_t)l + hmax;
    int hb = 1;
    while (hb < 31 && (1ull << hb) <= hsum) hb++;
    const bool narrow = hb < 31 && ((2ull * wmax + 1) << hb) <= (1ull << 30);
    if ((double)nnz >= (narrow ? kDenseFracNarrow : kDenseFracWide) * (double)total) {
      ProfScope ps(c, narrow ? "apsp.dense_round.u32" : "apsp.dense_round.u64", 8.0 * 3.0 * (double)total, s);
      const uint32_t l2 = (uint32_t)std::min<int64_t>(2 * l, 0xffffffffll);
      int64_t *nc = 2 * l < n ? cnt.as<int64_t>() : nullptr;  // counts for the next round
      if (nc) fill_i64(nc, n, 0, s);
      const dim3 grid((unsigned)((n + DTN - 1) / DTN), (unsigned)((n + DTM - 1) / DTM));
      if (narrow) {
        // 64 x 64 tiles, 3 blocks per CU: measured best at n = 2048 of
        // 128x128 (k 16/32), 128x64, 64x128 (k 32/64) and 64x64 (k 32/64)
        apsp_dense_round<Narrow, DTM, DTN, DTK, 3><<<grid, 256, 0, s>>>(
            P, Pn, n, (uint32_t)l, (uint32_t)idw, Narrow{(uint32_t)idw, hb}, nc, l2, part.as<uint32_t>());
      } else {
        apsp_dense_round<Wide, DTM, DTN, 16, 2><<<grid, 256, 0, s>>>(P, Pn, n, (uint32_t)l, (uint32_t)idw,
                                                                      Wide{idv}, nc, l2, part.as<uint32_t>());
      }
      counted = nc != nullptr;
      SRTC_LAUNCH_CHECK("apsp_dense_round");
      c->tracef("apsp: dense round, %s values (hop bits %d)", narrow ? "32-bit" : "64-bit", hb);
      std::swap(P, Pn);
      r++;
      continue;
    }
    Buf pc(c, sizeof(int32_t) * (size_t)nnz), pv(c, sizeof(uint64_t) * (size_t)nnz);
    {
      ProfScope ps(c, "apsp.hops_fill", 8.0 * (double)total + 12.0 * (double)nnz, s);
      hops_fill<<<grid_of(n * WAVE), 256, 0, s>>>(P, n, (uint32_t)l, (uint32_t)idw, rp.as<int64_t>(),
                                                   pc.as<int32_t>(), pv.as<uint64_t>());
    }
    SRTC_LAUNCH_CHECK("hops_fill");
    CsrView pl;
    pl.m = n;
    pl.n = n;
    pl.nnz = nnz;
    pl.rowptr = rp.as<int64_t>();
    pl.col = pc.as<int32_t>();
    pl.val = pv.p;
    SRTC_HIP(hipMemcpyAsync(Pn, P, sizeof(uint64_t) * (size_t)total, hipMemcpyDeviceToDevice, s));
    spmm(c, SRTC_MIN_PLUS, SRTC_PATH64, id, pl, P, n, Pn, 1, s);  // Pn = P (+) Pl (x) P
    std::swap(P, Pn);
    counted = false;
    r++;
  }
  if (total > 0) {
    ProfScope ps(c, "apsp.out", (H ? 16.0 : 12.0) * (double)total, s);
    apsp_out<<<grid_of(total), 256, 0, s>>>(P, total, (uint32_t)idw, D, H);
    SRTC_LAUNCH_CHECK("apsp_out");
  }
  if (rounds) *rounds = r;
}

}  // namespace srtc
