// Hub tiles: the dense corner of a power-law product on the matrix cores.
//
// The paper's local kernels favour small dense blocks where the data has
// them (Section 6.2).  In a power-law graph the highest-degree vertices
// ("hubs") form such a block: with H_i the hub rows of A, H_k the hub inner
// indices and H_j the hub columns of B,
//
//   A (x) B = A_x (x) B  (+)  A_h (x) B_x  (+)  A_h (x) B_hh
//
// where A_h holds A's entries in H_i x H_k and A_x the rest of A, B_hh holds
// B's entries in H_k x H_j and B_x the rest of B's rows in H_k (A_h has no
// other columns, so no other row of B meets it).  D = A_h (x) B_hh is formed
// as one dense |H_i| x |H_k| by |H_k| x |H_j| product on the MFMA tile, its
// nonzeros become a sparse matrix over C's rows, and the three terms are one
// sparse product over augmented operands,
//
//   [A_x | A_h | I] (x) [B ; B_x ; D],
//
// whose inner index runs over B's rows, then B_x's, then D's (the identity
// entry of row i picks D's row i as one more term of row i's sum).  Only the
// (+,x) semiring qualifies: a zero of the dense tile is its additive
// identity, so absent entries and zero products coincide.
//
// Hubs are chosen on the device: each index set is the |H| indices with the
// most entries (rows of A by row length, inner indices by A's column count
// plus B's row length, columns of B by column count), ties to the smaller
// index, then listed in ascending order (so D's rows list columns in order).
#include <algorithm>

#include "internal.hpp"

namespace srtc {

namespace {

inline unsigned gridn(int64_t n, int bs = 256, int64_t cap = 65536) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + bs - 1) / bs, cap));
}

__global__ void row_lengths(const int64_t *__restrict__ rp, int64_t m, uint32_t *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint32_t)std::min<int64_t>(rp[i + 1] - rp[i], 0xffffffffll);
}

// out[col] += 1 per entry (out starts at `init`, or zero)
__global__ void col_counts(const int64_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t m,
                           uint32_t *__restrict__ out) {
  const int64_t b = rp[0], e = rp[m];
  for (int64_t q = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < e; q += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&out[col[q]], 1u);
}

// sort keys: larger score first (stable sort keeps smaller indices first)
__global__ void score_keys(const uint32_t *__restrict__ score, int64_t n, int64_t *__restrict__ keys,
                           uint32_t *__restrict__ idx) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    keys[v] = (int64_t)(0xffffffffu - score[v]);
    idx[v] = (uint32_t)v;
  }
}

__global__ void mark_first(const uint32_t *__restrict__ idx, int64_t k, int32_t *__restrict__ flag) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < k; r += (int64_t)gridDim.x * blockDim.x)
    flag[idx[r]] = 1;
}

// pos = exclusive scan of flag: hub v gets slot pos[v]; others -1
__global__ void hub_slots(const int32_t *__restrict__ flag, const int64_t *__restrict__ pos, int64_t n,
                          int32_t *__restrict__ slot, int32_t *__restrict__ ids) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (flag[v]) {
      slot[v] = (int32_t)pos[v];
      ids[pos[v]] = (int32_t)v;
    } else {
      slot[v] = -1;
    }
  }
}

// dense[hr[i] * ncols + hc[col]] = value for the entries of hub rows in hub
// columns (one wave per row; entries of one row have distinct columns)
template <class V>
__global__ void fill_tile(const int64_t *__restrict__ rp, const int32_t *__restrict__ col, const V *__restrict__ val,
                          int64_t m, const int32_t *__restrict__ hr, const int32_t *__restrict__ hc, int64_t ncols,
                          V *__restrict__ dense) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t i = wid; i < m; i += nw) {
    const int32_t r = hr[i];
    if (r < 0) continue;
    for (int64_t q = rp[i] + lane_id(); q < rp[i + 1]; q += WAVE) {
      const int32_t c = hc[col[q]];
      if (c >= 0) dense[(int64_t)r * ncols + c] = val[q];
    }
  }
}

// nonzeros of each row of the dense product, placed at the hub row's index
template <class V>
__global__ void tile_row_counts(const V *__restrict__ D, int64_t ki, int64_t kj, const int32_t *__restrict__ hi_ids,
                                int64_t *__restrict__ cnt) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t r = wid; r < ki; r += nw) {
    int64_t n = 0;
    for (int64_t c0 = 0; c0 < kj; c0 += WAVE) {
      const int64_t c = c0 + lane_id();
      n += __popcll(__ballot(c < kj && D[r * kj + c] != V(0)));
    }
    if (lane_id() == 0) cnt[hi_ids[r]] = n;
  }
}

// the dense product's nonzeros as CSR entries over C's rows and columns
template <class V>
__global__ void tile_row_entries(const V *__restrict__ D, int64_t ki, int64_t kj, const int32_t *__restrict__ hi_ids,
                                 const int32_t *__restrict__ hj_ids, const int64_t *__restrict__ rpD,
                                 int32_t *__restrict__ colD, V *__restrict__ valD) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  const uint64_t lt = lanemask_lt();
  for (int64_t r = wid; r < ki; r += nw) {
    int64_t o = rpD[hi_ids[r]];
    for (int64_t c0 = 0; c0 < kj; c0 += WAVE) {
      const int64_t c = c0 + lane_id();
      const V v = c < kj ? D[r * kj + c] : V(0);
      const bool keep = v != V(0);
      const uint64_t mk = __ballot(keep);
      if (keep) {
        const int64_t p = o + __popcll(mk & lt);
        colD[p] = hj_ids[c];
        valD[p] = v;
      }
      o += __popcll(mk);
    }
  }
}

// Row lengths of the augmented A: hub rows get one identity entry.
__global__ void aug_rows_a(const int64_t *__restrict__ rpA, int64_t m, const int32_t *__restrict__ hr,
                           int64_t *__restrict__ len) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    len[i] = rpA[i + 1] - rpA[i] + (hr[i] >= 0 ? 1 : 0);
}

// Ordered compaction of one row's entries by a predicate (one wave): writes
// the kept entries from `o` on with columns + shift; returns the new `o`.
template <class V, class P>
__device__ __forceinline__ int64_t copy_if(const int32_t *__restrict__ col, const V *__restrict__ val, int64_t b,
                                           int64_t e, int64_t shift, int64_t o, int32_t *__restrict__ ocol,
                                           V *__restrict__ oval, P &&pred) {
  const uint64_t lt = lanemask_lt();
  for (int64_t q0 = b; q0 < e; q0 += WAVE) {
    const int64_t q = q0 + lane_id();
    const bool keep = q < e && pred(col[q]);
    const uint64_t mk = __ballot(keep);
    if (keep) {
      const int64_t p = o + __popcll(mk & lt);
      ocol[p] = (int32_t)(col[q] + shift);
      oval[p] = val[q];
    }
    o += __popcll(mk);
  }
  return o;
}

// [A_x | A_h | I]: row i lists its entries outside H_i x H_k (columns k),
// then those inside (columns n + k), then, for a hub row, the identity entry
// (column 2n + i); the three blocks keep the row ascending.
template <class V>
__global__ void aug_entries_a(const int64_t *__restrict__ rpA, const int32_t *__restrict__ cA,
                              const V *__restrict__ vA, int64_t m, int64_t n, const int32_t *__restrict__ hr,
                              const int32_t *__restrict__ hk, V one, const int64_t *__restrict__ rp,
                              int32_t *__restrict__ col, V *__restrict__ val) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t i = wid; i < m; i += nw) {
    const int64_t b = rpA[i], e = rpA[i + 1];
    int64_t o = rp[i];
    if (hr[i] < 0) {
      for (int64_t q = b + lane_id(); q < e; q += WAVE) {
        col[o + q - b] = cA[q];
        val[o + q - b] = vA[q];
      }
      continue;
    }
    o = copy_if(cA, vA, b, e, 0, o, col, val, [&](int32_t k) { return hk[k] < 0; });
    o = copy_if(cA, vA, b, e, n, o, col, val, [&](int32_t k) { return hk[k] >= 0; });
    if (lane_id() == 0) {
      col[o] = (int32_t)(2 * n + i);
      val[o] = one;
    }
  }
}

// Row lengths of [B ; B_x ; D]: B's rows, then B's hub rows without hub
// columns (other rows empty), then D's rows.
__global__ void aug_rows_b(const int64_t *__restrict__ rpB, const int32_t *__restrict__ cB, int64_t n,
                           const int32_t *__restrict__ hk, const int32_t *__restrict__ hj,
                           const int64_t *__restrict__ rpD, int64_t m, int64_t *__restrict__ len) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t r = wid; r < 2 * n + m; r += nw) {
    int64_t v = 0;
    if (r < n) {
      v = rpB[r + 1] - rpB[r];
    } else if (r < 2 * n) {
      const int64_t k = r - n;
      if (hk[k] >= 0) {
        for (int64_t q = rpB[k] + lane_id(); q < rpB[k + 1]; q += WAVE) v += hj[cB[q]] < 0 ? 1 : 0;
        v = wave_sum(v);
      }
    } else {
      v = rpD[r - 2 * n + 1] - rpD[r - 2 * n];
    }
    if (lane_id() == 0) len[r] = v;
  }
}

template <class V>
__global__ void aug_entries_b(const int64_t *__restrict__ rpB, const int32_t *__restrict__ cB,
                              const V *__restrict__ vB, int64_t n, const int32_t *__restrict__ hk,
                              const int32_t *__restrict__ hj, const int64_t *__restrict__ rpD,
                              const int32_t *__restrict__ cD, const V *__restrict__ vD, int64_t m,
                              const int64_t *__restrict__ rp, int32_t *__restrict__ col, V *__restrict__ val) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t r = wid; r < 2 * n + m; r += nw) {
    const int64_t o = rp[r];
    if (r < n) {
      const int64_t b = rpB[r], e = rpB[r + 1];
      for (int64_t q = b + lane_id(); q < e; q += WAVE) {
        col[o + q - b] = cB[q];
        val[o + q - b] = vB[q];
      }
    } else if (r < 2 * n) {
      const int64_t k = r - n;
      if (hk[k] >= 0) copy_if(cB, vB, rpB[k], rpB[k + 1], 0, o, col, val, [&](int32_t j) { return hj[j] < 0; });
    } else {
      const int64_t i = r - 2 * n, b = rpD[i], e = rpD[i + 1];
      for (int64_t q = b + lane_id(); q < e; q += WAVE) {
        col[o + q - b] = cD[q];
        val[o + q - b] = vD[q];
      }
    }
  }
}

// The `k` indices of [0, n) with the largest scores, as slot[v] (position
// among them in ascending order, -1 for others) and ids[0..k) ascending.
void pick_hubs(Ctx *c, const uint32_t *score, int64_t n, int64_t k, int32_t *slot, int32_t *ids, hipStream_t s) {
  Buf keys(c, sizeof(int64_t) * (size_t)n), idx(c, sizeof(uint32_t) * (size_t)n);
  Buf flag(c, sizeof(int32_t) * (size_t)n), pos(c, sizeof(int64_t) * (size_t)(n + 1));
  score_keys<<<gridn(n), 256, 0, s>>>(score, n, keys.as<int64_t>(), idx.as<uint32_t>());
  SRTC_LAUNCH_CHECK("score_keys");
  radix_sort_pairs(c, keys.as<int64_t>(), idx.as<uint32_t>(), n, 32, s);
  fill_i32(flag.as<int32_t>(), n, 0, s);
  mark_first<<<gridn(k), 256, 0, s>>>(idx.as<uint32_t>(), k, flag.as<int32_t>());
  SRTC_LAUNCH_CHECK("mark_first");
  excl_scan_i32(c, flag.as<int32_t>(), pos.as<int64_t>(), n, s);
  hub_slots<<<gridn(n), 256, 0, s>>>(flag.as<int32_t>(), pos.as<int64_t>(), n, slot, ids);
  SRTC_LAUNCH_CHECK("hub_slots");
}

template <class V>
void hub_product_typed(Ctx *c, int dt, IdVal id, const CsrView &A, const CsrView &B, int64_t hub, int sched,
                       int sorted, CsrOut *out, SpgemmStats *st, hipStream_t s) {
  const int64_t m = A.m, n = A.n, nc = B.n;
  const int64_t ki = std::min(hub, m), kk = std::min(hub, n), kj = std::min(hub, nc);
  // hub sets
  Buf sr(c, sizeof(uint32_t) * (size_t)m), sk(c, sizeof(uint32_t) * (size_t)n), sj(c, sizeof(uint32_t) * (size_t)nc);
  Buf hr(c, sizeof(int32_t) * (size_t)m), hk(c, sizeof(int32_t) * (size_t)n), hj(c, sizeof(int32_t) * (size_t)nc);
  Buf ir(c, sizeof(int32_t) * (size_t)ki), ik(c, sizeof(int32_t) * (size_t)kk), ij(c, sizeof(int32_t) * (size_t)kj);
  {
    ProfScope ps(c, "spgemm.hub_select", 8.0 * (A.nnz + B.nnz) + 12.0 * (m + n + nc), s);
    row_lengths<<<gridn(m), 256, 0, s>>>(A.rowptr, m, sr.as<uint32_t>());
    SRTC_LAUNCH_CHECK("row_lengths");
    row_lengths<<<gridn(n), 256, 0, s>>>(B.rowptr, n, sk.as<uint32_t>());
    SRTC_LAUNCH_CHECK("row_lengths");
    col_counts<<<gridn(A.nnz, 256, 16384), 256, 0, s>>>(A.rowptr, A.col, m, sk.as<uint32_t>());
    SRTC_LAUNCH_CHECK("col_counts");
    fill_i32(reinterpret_cast<int32_t *>(sj.p), nc, 0, s);
    col_counts<<<gridn(B.nnz, 256, 16384), 256, 0, s>>>(B.rowptr, B.col, n, sj.as<uint32_t>());
    SRTC_LAUNCH_CHECK("col_counts");
    pick_hubs(c, sr.as<uint32_t>(), m, ki, hr.as<int32_t>(), ir.as<int32_t>(), s);
    pick_hubs(c, sk.as<uint32_t>(), n, kk, hk.as<int32_t>(), ik.as<int32_t>(), s);
    pick_hubs(c, sj.as<uint32_t>(), nc, kj, hj.as<int32_t>(), ij.as<int32_t>(), s);
  }
  // D = A_h (x) B_hh on the matrix cores
  Buf ta(c, sizeof(V) * (size_t)(ki * kk)), tb(c, sizeof(V) * (size_t)(kk * kj)), td(c, sizeof(V) * (size_t)(ki * kj));
  {
    ProfScope ps(c, "spgemm.hub_tiles", (double)sizeof(V) * (double)(ki * kk + kk * kj) + 12.0 * (A.nnz + B.nnz), s);
    fill_bytes_value(ta.p, ki * kk, dt, IdVal{}, s);
    fill_bytes_value(tb.p, kk * kj, dt, IdVal{}, s);
    fill_tile<V><<<gridn(m * WAVE), 256, 0, s>>>(A.rowptr, A.col, (const V *)A.val, m, hr.as<int32_t>(),
                                                  hk.as<int32_t>(), kk, ta.as<V>());
    SRTC_LAUNCH_CHECK("fill_tile");
    fill_tile<V><<<gridn(n * WAVE), 256, 0, s>>>(B.rowptr, B.col, (const V *)B.val, n, hk.as<int32_t>(),
                                                  hj.as<int32_t>(), kj, tb.as<V>());
    SRTC_LAUNCH_CHECK("fill_tile");
  }
  {
    ProfScope ps(c, dt == SRTC_F64 ? "spgemm.hub_gemm_mfma.f64" : "spgemm.hub_gemm_mfma.f32",
                 (double)sizeof(V) * (double)(ki * kk + kk * kj + ki * kj), s);
    dense_gemm_plus_times(c, dt, ta.p, tb.p, td.p, ki, kj, kk, 0, s);
  }
  // D's nonzeros over C's rows
  Buf dcnt(c, sizeof(int64_t) * (size_t)m), rpD(c, sizeof(int64_t) * (size_t)(m + 1));
  fill_i64(dcnt.as<int64_t>(), m, 0, s);
  tile_row_counts<V><<<gridn(ki * WAVE), 256, 0, s>>>(td.as<V>(), ki, kj, ir.as<int32_t>(), dcnt.as<int64_t>());
  SRTC_LAUNCH_CHECK("tile_row_counts");
  excl_scan_i64(c, dcnt.as<int64_t>(), rpD.as<int64_t>(), m, s);
  const int64_t nD = read_i64(c, rpD.as<int64_t>() + m, s);
  Buf cD(c, sizeof(int32_t) * (size_t)std::max<int64_t>(nD, 1)), vD(c, sizeof(V) * (size_t)std::max<int64_t>(nD, 1));
  tile_row_entries<V><<<gridn(ki * WAVE), 256, 0, s>>>(td.as<V>(), ki, kj, ir.as<int32_t>(), ij.as<int32_t>(),
                                                        rpD.as<int64_t>(), cD.as<int32_t>(), vD.as<V>());
  SRTC_LAUNCH_CHECK("tile_row_entries");
  ta = Buf();
  tb = Buf();
  td = Buf();
  // the augmented operands
  Buf lenA(c, sizeof(int64_t) * (size_t)m), rpA2(c, sizeof(int64_t) * (size_t)(m + 1));
  const int64_t nB2rows = 2 * n + m;
  Buf lenB(c, sizeof(int64_t) * (size_t)nB2rows), rpB2(c, sizeof(int64_t) * (size_t)(nB2rows + 1));
  Buf cA2, vA2, cB2, vB2;
  int64_t nA2 = A.nnz + ki, nB2 = 0;
  {
    ProfScope ps(c, "spgemm.hub_operands", 24.0 * (A.nnz + B.nnz) + 12.0 * nD, s);
    aug_rows_a<<<gridn(m), 256, 0, s>>>(A.rowptr, m, hr.as<int32_t>(), lenA.as<int64_t>());
    SRTC_LAUNCH_CHECK("aug_rows_a");
    excl_scan_i64(c, lenA.as<int64_t>(), rpA2.as<int64_t>(), m, s);
    cA2 = Buf(c, sizeof(int32_t) * (size_t)std::max<int64_t>(nA2, 1));
    vA2 = Buf(c, sizeof(V) * (size_t)std::max<int64_t>(nA2, 1));
    aug_entries_a<V><<<gridn(m * WAVE), 256, 0, s>>>(A.rowptr, A.col, (const V *)A.val, m, n, hr.as<int32_t>(),
                                                      hk.as<int32_t>(), V(1), rpA2.as<int64_t>(), cA2.as<int32_t>(),
                                                      vA2.as<V>());
    SRTC_LAUNCH_CHECK("aug_entries_a");
    aug_rows_b<<<gridn(nB2rows * WAVE), 256, 0, s>>>(B.rowptr, B.col, n, hk.as<int32_t>(), hj.as<int32_t>(),
                                                      rpD.as<int64_t>(), m, lenB.as<int64_t>());
    SRTC_LAUNCH_CHECK("aug_rows_b");
    excl_scan_i64(c, lenB.as<int64_t>(), rpB2.as<int64_t>(), nB2rows, s);
    nB2 = read_i64(c, rpB2.as<int64_t>() + nB2rows, s);
    cB2 = Buf(c, sizeof(int32_t) * (size_t)std::max<int64_t>(nB2, 1));
    vB2 = Buf(c, sizeof(V) * (size_t)std::max<int64_t>(nB2, 1));
    aug_entries_b<V><<<gridn(nB2rows * WAVE), 256, 0, s>>>(B.rowptr, B.col, (const V *)B.val, n, hk.as<int32_t>(),
                                                            hj.as<int32_t>(), rpD.as<int64_t>(), cD.as<int32_t>(),
                                                            vD.as<V>(), m, rpB2.as<int64_t>(), cB2.as<int32_t>(),
                                                            vB2.as<V>());
    SRTC_LAUNCH_CHECK("aug_entries_b");
  }
  const CsrView A2{m, nB2rows, nA2, rpA2.as<int64_t>(), cA2.as<int32_t>(), vA2.p};
  const CsrView B2{nB2rows, nc, nB2, rpB2.as<int64_t>(), cB2.as<int32_t>(), vB2.p};
  spgemm(c, SRTC_PLUS_TIMES, dt, id, A2, B2, sched, sorted, out, st, s);
}

}  // namespace

bool hub_product_applies(int sr, int dt, const CsrView &A, const CsrView &B, int64_t hub) {
  return hub > 0 && sr == SRTC_PLUS_TIMES && (dt == SRTC_F64 || dt == SRTC_F32) && A.m > 0 && A.n > 0 && B.n > 0 &&
         2 * A.n + A.m < 0x7fffffffll && B.n < 0x7fffffffll;
}

void spgemm_hubs(Ctx *c, int dt, IdVal id, const CsrView &A, const CsrView &B, int64_t hub, int sched, int sorted,
                 CsrOut *out, SpgemmStats *st, hipStream_t s) {
  if (dt == SRTC_F64)
    hub_product_typed<double>(c, dt, id, A, B, hub, sched, sorted, out, st, s);
  else if (dt == SRTC_F32)
    hub_product_typed<float>(c, dt, id, A, B, hub, sched, sorted, out, st, s);
  else
    fail(SRTC_ERR_DTYPE, "hub tiles: (+,x) on F64 or F32 only");
}

}  // namespace srtc
