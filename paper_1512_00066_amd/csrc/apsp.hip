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

// One thread per row, so repeated entries of a row combine without atomics.
__global__ void apsp_edges(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const int32_t *__restrict__ w, int64_t n, int32_t idw, uint64_t *__restrict__ P,
                           int32_t *bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
      const int32_t x = w[p];
      if (x < 0) {
        atomicOr(bad, 1);
        continue;
      }
      if (x >= idw) continue;
      const uint64_t v = ((uint64_t)(uint32_t)x << 32) | 1ull;
      uint64_t *cell = P + i * n + col[p];
      if (v < *cell) *cell = v;
    }
  }
}

// Entries of row i whose path has exactly l hops (wave per row).
__global__ void hops_count(const uint64_t *__restrict__ P, int64_t n, uint32_t l, uint32_t idw,
                           int64_t *__restrict__ cnt) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t i = wid; i < n; i += nw) {
    int64_t c = 0;
    for (int64_t j = lane_id(); j < n; j += WAVE) {
      const uint64_t v = P[i * n + j];
      c += ((uint32_t)v == l && (uint32_t)(v >> 32) < idw) ? 1 : 0;
    }
    c = wave_sum(c);
    if (lane_id() == 0) cnt[i] = c;
  }
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
void apsp_tiskin(Ctx *c, const CsrView &A, int32_t idw, int32_t *D, int32_t *H, int32_t *rounds, int64_t *round_nnz,
                 hipStream_t s) {
  const int64_t n = A.m;
  if (A.n != n) fail(SRTC_ERR_DIM, "apsp: A must be square");
  if (n > 0xffffffffll / 2) fail(SRTC_ERR_UNSUPPORTED, "apsp: too many vertices");
  if ((uint64_t)n * (uint64_t)n > (1ull << 40)) fail(SRTC_ERR_UNSUPPORTED, "apsp: dense n x n path matrix too large");
  const uint64_t idv = (uint64_t)(uint32_t)idw << 32;
  const int64_t total = n * n;
  Buf pa(c, sizeof(uint64_t) * (size_t)std::max<int64_t>(total, 1)), pb(c, sizeof(uint64_t) * (size_t)std::max<int64_t>(total, 1));
  Buf bad(c, 64);
  fill_i32(bad.as<int32_t>(), 1, 0, s);
  uint64_t *P = pa.as<uint64_t>(), *Pn = pb.as<uint64_t>();
  apsp_init<<<grid_of(total), 256, 0, s>>>(P, n, idv);
  SRTC_LAUNCH_CHECK("apsp_init");
  if (A.nnz > 0) {
    apsp_edges<<<grid_of(n), 256, 0, s>>>(A.rowptr, A.col, (const int32_t *)A.val, n, idw, P, bad.as<int32_t>());
    SRTC_LAUNCH_CHECK("apsp_edges");
  }
  int32_t neg = 0;
  read_to_host(c, &neg, bad.p, sizeof(neg), s);
  if (neg) fail(SRTC_ERR_ARG, "apsp: negative edge weight");
  const IdVal id{0.0, (int64_t)idw};
  Buf cnt(c, sizeof(int64_t) * (size_t)std::max<int64_t>(n, 1)), rp(c, sizeof(int64_t) * (size_t)(n + 1));
  int32_t r = 0;
  if (round_nnz) std::fill(round_nnz, round_nnz + 64, (int64_t)0);
  for (int64_t l = 1; l < n; l <<= 1) {
    hops_count<<<grid_of(n * WAVE), 256, 0, s>>>(P, n, (uint32_t)l, (uint32_t)idw, cnt.as<int64_t>());
    SRTC_LAUNCH_CHECK("hops_count");
    excl_scan_i64(c, cnt.as<int64_t>(), rp.as<int64_t>(), n, s);
    const int64_t nnz = read_i64(c, rp.as<int64_t>() + n, s);
    c->tracef("apsp: round %d, %lld paths of %lld hops", r, (long long)nnz, (long long)l);
    if (round_nnz && r < 64) round_nnz[r] = nnz;
    if (nnz == 0) break;  // no path has more than l hops
    Buf pc(c, sizeof(int32_t) * (size_t)nnz), pv(c, sizeof(uint64_t) * (size_t)nnz);
    hops_fill<<<grid_of(n * WAVE), 256, 0, s>>>(P, n, (uint32_t)l, (uint32_t)idw, rp.as<int64_t>(), pc.as<int32_t>(),
                                                 pv.as<uint64_t>());
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
    r++;
  }
  if (total > 0) {
    apsp_out<<<grid_of(total), 256, 0, s>>>(P, total, (uint32_t)idw, D, H);
    SRTC_LAUNCH_CHECK("apsp_out");
  }
  if (rounds) *rounds = r;
}

}  // namespace srtc
