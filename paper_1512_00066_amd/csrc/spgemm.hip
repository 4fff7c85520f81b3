// Sparse x sparse semiring contraction C = A (x) B (row-wise, two phases).
//
//   C_ij = (+)_{k : (i,k) in A, (k,j) in B} A_ik (x) B_kj
// (the loop-nest meaning of an indexed contraction, Section 3.3.1; sparse x
// sparse is the extension left open in Sections 1 and 7).
//
// Pipeline (all rows of A are independent):
//   1. row analysis   w_i = sum_{k in A_i} nnz(B_k)   (products per row)
//   2. binning        rows grouped by w_i, then by the exact nnz_i
//   3. symbolic       nnz_i per row: LDS hash of column keys (light rows) or
//                     an LDS bitmap over the columns (heavy rows)
//   4. scan           rowptr of C; the single host sync sizes C
//   5. numeric        per bin: LDS hash, then the kept entries placed by
//                     rank or bitonic-sorted in LDS, or dense LDS
//                     accumulator windows and ranked groups over the columns
//                     (heavy rows)
//   6. compaction     only if some result equalled the additive identity
//                     (dropped, or written with column -1), the rows are
//                     packed again.
// Every per-bin kernel is persistent: a grid sized to the machine pulls rows
// from an atomic work counter.
#include <algorithm>
#include <cmath>
#include <vector>

#include <string>
#include <type_traits>

#include "internal.hpp"

namespace srtc {

namespace {

constexpr int32_t EMPTY = 0x7fffffff;  // empty hash slot (sorts last)

// Where a row's output goes: entries start[i] .. start[i] + count[i] - 1 of
// C's arrays, columns shifted by col_off (a column block of B carries
// block-local columns).
struct OutRows {
  const int64_t *start;
  const int64_t *count;
  int64_t col_off;
};
constexpr int LDS_BYTES = 160 * 1024;

__device__ __forceinline__ uint32_t hash_slot(int32_t j, int lg) {
  return ((uint32_t)j * 0x9E3779B1u) >> (32 - lg);
}

// ------------------------------------------------------------- analysis --
__global__ void row_products_kernel(const int64_t *__restrict__ rpA, const int32_t *__restrict__ cA,
                                    const int64_t *__restrict__ rpB, int64_t m, int64_t *__restrict__ w) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t i = wid; i < m; i += nw) {
    int64_t acc = 0;
    for (int64_t p = rpA[i] + lane_id(); p < rpA[i + 1]; p += WAVE) {
      const int32_t k = cA[p];
      acc += rpB[k + 1] - rpB[k];
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) w[i] = acc;
  }
}

constexpr int NBIN = 6;  // bin 0 = empty rows (skipped)
struct Thresholds {
  int64_t t[NBIN - 1];  // bin b (1..) takes v with t[b-2] < v <= t[b-1]; last bin above
};

// info layout: [0..NBIN) counts, [NBIN..2NBIN) starts, [2NBIN..3NBIN) cursors,
// [3NBIN..4NBIN) work counters, [4NBIN] sum of values, [SUMV..SUMV+NBIN)
// per-bin sums of values, [SUMA..SUMA+NBIN) per-bin sums of A row lengths
constexpr int SUMV = 4 * NBIN + 1;
constexpr int SUMA = 5 * NBIN + 1;
constexpr int INFO = 6 * NBIN + 2;

__device__ __forceinline__ int bin_of(int64_t v, const Thresholds &th) {
  if (v <= 0) return 0;
#pragma unroll
  for (int b = 0; b < NBIN - 2; b++)
    if (v <= th.t[b]) return b + 1;
  return NBIN - 1;
}

__global__ void bin_count(const int64_t *v, int64_t m, Thresholds th, int64_t *info, const int64_t *rpA,
                          const int32_t *row_map) {
  __shared__ int32_t cnt[NBIN];
  __shared__ unsigned long long sv[NBIN], sa[NBIN];
  __shared__ unsigned long long sum;
  if (threadIdx.x < NBIN) { cnt[threadIdx.x] = 0; sv[threadIdx.x] = 0; sa[threadIdx.x] = 0; }
  if (threadIdx.x == 0) sum = 0;
  __syncthreads();
  unsigned long long local = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = v[i];
    const int b = bin_of(x, th);
    const int64_t r = row_map ? row_map[i] : i;
    atomicAdd(&cnt[b], 1);
    atomicAdd(&sv[b], (unsigned long long)x);
    atomicAdd(&sa[b], (unsigned long long)(rpA[r + 1] - rpA[r]));
    local += (unsigned long long)x;
  }
  local = wave_sum(local);
  if (lane_id() == 0) atomicAdd(&sum, local);
  __syncthreads();
  if (threadIdx.x < NBIN) {
    atomicAdd((unsigned long long *)&info[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
    atomicAdd((unsigned long long *)&info[SUMV + threadIdx.x], sv[threadIdx.x]);
    atomicAdd((unsigned long long *)&info[SUMA + threadIdx.x], sa[threadIdx.x]);
  }
  if (threadIdx.x == 0) atomicAdd((unsigned long long *)&info[4 * NBIN], sum);
}

__global__ void bin_offsets(int64_t *info) {
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int b = 0; b < NBIN; b++) {
      info[NBIN + b] = run;
      info[2 * NBIN + b] = 0;
      info[3 * NBIN + b] = 0;
      run += info[b];
    }
  }
}

// Rows go to their bin's list; each wave takes one slot range per bin with a
// single atomic and places its rows by ballot rank.
__global__ void bin_scatter(const int64_t *v, int64_t m, Thresholds th, int64_t *info, int32_t *lists,
                            const int32_t *row_map) {
  const uint64_t lt = lanemask_lt();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < m; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    const int b = i < m ? bin_of(v[i], th) : 0;
#pragma unroll
    for (int bb = 1; bb < NBIN; bb++) {
      const uint64_t mk = __ballot(b == bb);
      if (mk == 0) continue;
      const int leader = __ffsll((unsigned long long)mk) - 1;
      long long p = 0;
      if (lane_id() == leader)
        p = (long long)atomicAdd((unsigned long long *)&info[2 * NBIN + bb], (unsigned long long)__popcll(mk));
      p = __shfl(p, leader, WAVE);
      if (b == bb) lists[info[NBIN + bb] + p + __popcll(mk & lt)] = row_map ? row_map[i] : (int32_t)i;
    }
  }
}

// Sort key putting heavy rows first: descending in a 16-bit code of the
// row's product count (exponent and three mantissa bits).
__global__ void heavy_first_keys(const int32_t *__restrict__ rows, const int64_t *__restrict__ w, int64_t n,
                                 int64_t *__restrict__ keys) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t x = (uint64_t)max((int64_t)1, w[rows[q]]);
    const int e = 63 - __clzll(x);
    const uint64_t mant = e >= 3 ? (x >> (e - 3)) & 7 : (x << (3 - e)) & 7;
    keys[q] = 0xFFFF - (int64_t)(e * 8 + mant);
  }
}

__global__ void gather_i64(const int64_t *src, const int32_t *idx, int64_t n, int64_t *dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[idx[i]];
}

// ------------------------------------------------------ product walking --
template <int BS, class V> struct Chunk {
  int32_t off[BS];
  int64_t start[BS];
  V a[BS];
  int32_t tmp[BS / WAVE + 1];
};

// Walking the products laid out by a chunk: L.off holds the exclusive scan of
// the cnt segment lengths (total products), L.start each segment's first
// position in B, L.a the A value.  The products are taken in tiles of BS*U;
// in a tile, thread t takes U consecutive ones, t*U .. t*U+U-1.  A binary
// search finds the segment owning the first; the next ones advance from it
// (one comparison with the next segment's offset, the B position otherwise
// just increments), so the search is paid once per batch of U products, not
// per product, and a lane keeps U independent loads in flight.  Gathering a
// batch and consuming it are separate steps, so a caller can issue the loads
// early and use them later.  REC: B's entries are read from rB, (column,
// value) records, instead of the two arrays.  For 8-byte values a batch
// keeps each product's A entry (its segment in the layout) rather than the A
// value, read from the layout when the batch is consumed: two registers per
// product fewer (the fp64 dense-window kernel 1.8% faster; for 4-byte values
// the extra LDS reads cost more than the registers save).
template <int U, class V> struct Batch {
  static constexpr bool IDX = sizeof(V) == 8;
  int32_t j[U];
  std::conditional_t<IDX, int32_t, V> a[U];
  V b[U];
};

// B entries of semirings with 4-byte values as 8-byte (column, value bits)
// records: a product's column and value then come from one cache line.  In
// the dense windows most B segments are shorter than a line, so with the two
// arrays a product touched two lines.  (For 8-byte values, 12- and 16-byte
// records measured slower than the two arrays.)
template <class SR> constexpr bool b_records() {
  return SR::HAS_VALS && sizeof(typename SR::val_t) == 4;
}

// r[i] = entry rowptr[0] + i of B, for the n = nnz entries of the view (the
// row pointers of a view into a larger matrix need not start at 0)
template <class V>
__global__ void pack_records(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ c,
                             const V *__restrict__ v, int64_t n, uint2 *__restrict__ r) {
  static_assert(sizeof(V) == 4, "4-byte values");
  const int64_t lo = rowptr[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = make_uint2((uint32_t)c[lo + i], __builtin_bit_cast(uint32_t, v[lo + i]));
}

template <int BS, int U, bool VALS, class V, bool REC = false>
__device__ __forceinline__ void gather_batch(const int32_t *__restrict__ cB, const V *__restrict__ vB, int cnt,
                                             int32_t total, const Chunk<BS, V> &L, int32_t base, Batch<U, V> &g,
                                             const uint2 *__restrict__ rB = nullptr) {
  static_assert(!REC || (VALS && sizeof(V) == 4), "records hold 4-byte values");
  const int32_t q0 = base + (int32_t)threadIdx.x * U;
  // largest lo with off[lo] <= q0 (off is non-decreasing, off[0] = 0)
  int lo = 0;
  for (int step = cnt > 1 ? 1 << (31 - __clz(cnt - 1)) : 0; step > 0; step >>= 1) {
    const int c = lo + step;
    if (c < cnt && L.off[c] <= q0) lo = c;
  }
  int32_t nxt = lo + 1 < cnt ? L.off[lo + 1] : INT32_MAX;
  int64_t pos = L.start[lo] + (q0 - L.off[lo]);
  const int32_t *pc = REC ? nullptr : cB + pos;
  const V *pv = VALS && !REC ? vB + pos : nullptr;
  const uint2 *pr = REC ? rB + pos : nullptr;
  constexpr bool AV = VALS && !Batch<U, V>::IDX;  // the A value travels in the batch
  V av = AV ? L.a[lo] : V{};
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int32_t q = q0 + u;
    g.j[u] = 0;
    g.a[u] = {};
    g.b[u] = V{};
    if (q < total) {
      if (u > 0) {
        if (q >= nxt) {
          // the next non-empty segment (empty ones share its offset)
          do {
            lo++;
            nxt = lo + 1 < cnt ? L.off[lo + 1] : INT32_MAX;
          } while (q >= nxt);
          pos = L.start[lo] + (q - L.off[lo]);
          if constexpr (REC) {
            pr = rB + pos;
          } else {
            pc = cB + pos;
            if (VALS) pv = vB + pos;
          }
          if (AV) av = L.a[lo];
        } else if constexpr (REC) {
          pr++;
        } else {
          pc++;
          if (VALS) pv++;
        }
      }
      if constexpr (REC) {
        const uint2 e = *pr;
        g.j[u] = (int32_t)e.x;
        g.a[u] = av;  // records hold 4-byte values: the value itself
        g.b[u] = __builtin_bit_cast(V, e.y);
      } else {
        g.j[u] = *pc;
        if (VALS) {
          if constexpr (Batch<U, V>::IDX) g.a[u] = lo;
          else g.a[u] = av;
          g.b[u] = *pv;
        }
      }
    }
  }
}

// L: the layout the batch was gathered from (still in place).
template <int BS, int U, class V, class F>
__device__ __forceinline__ void consume_batch(const Batch<U, V> &g, const Chunk<BS, V> &L, int32_t base,
                                              int32_t total, F &&f) {
  const int32_t q0 = base + (int32_t)threadIdx.x * U;
#pragma unroll
  for (int u = 0; u < U; u++) {
    if (q0 + u >= total) continue;
    if constexpr (Batch<U, V>::IDX) f(g.j[u], L.a[g.a[u]], g.b[u]);
    else f(g.j[u], g.a[u], g.b[u]);
  }
}

// All products of a laid-out chunk from the tile starting at product `base`
// (a multiple of BS*U) on.  PIPE: the next tile's search and loads are
// issued before the current tile is consumed (twice the batch registers).
template <int BS, int U, bool VALS, class V, bool PIPE = false, bool REC = false, class F>
__device__ __forceinline__ void walk_chunk(const int32_t *__restrict__ cB, const V *__restrict__ vB, int cnt,
                                           int32_t total, const Chunk<BS, V> &L, F &&f, int32_t base = 0,
                                           const uint2 *__restrict__ rB = nullptr) {
  if constexpr (PIPE) {
    if (base >= total) return;
    Batch<U, V> g;
    gather_batch<BS, U, VALS, V, REC>(cB, vB, cnt, total, L, base, g, rB);
    for (int32_t b0 = base; b0 < total; b0 += BS * U) {
      Batch<U, V> h = g;
      if (b0 + BS * U < total) gather_batch<BS, U, VALS, V, REC>(cB, vB, cnt, total, L, b0 + BS * U, h, rB);
      consume_batch<BS, U, V>(g, L, b0, total, f);
      g = h;
    }
  } else {
    for (int32_t b0 = base; b0 < total; b0 += BS * U) {
      Batch<U, V> g;
      gather_batch<BS, U, VALS, V, REC>(cB, vB, cnt, total, L, b0, g, rB);
      consume_batch<BS, U, V>(g, L, b0, total, f);
    }
  }
}

constexpr int WALK_U = 4;
// products in flight per lane in the symbolic bitmap walk (column indices only)
constexpr int SYM_U = 4;

// Lay out one chunk's segments: thread t < cnt owns a segment of `len`
// products starting at B position `st` with A value `a`.  Returns the total;
// L is ready to walk when this returns.
template <int BS, bool VALS, class V>
__device__ __forceinline__ int32_t layout_chunk(int32_t len, int64_t st, V a, Chunk<BS, V> &L) {
  const int t = threadIdx.x;
  int32_t total;
  // the barrier below also orders these reads of L.tmp before its next use
  const int32_t off = block_excl_scan<BS, int32_t, false>(len, L.tmp, &total);
  L.off[t] = off;
  L.start[t] = st;
  if (VALS) L.a[t] = a;
  __syncthreads();
  return total;
}

// Visit every product of row i (optionally restricted to the column windows
// [w, w_end) of the window table) as f(j, a_ik, b_kj).  A entries are taken BS at a time;
// their B segments are laid end to end by a block scan and the threads walk
// that flattened range, so the work per thread is balanced whatever the
// segment lengths.
template <int BS, bool VALS, class V, int U = WALK_U, bool PIPE = false, bool REC = false, class F>
__device__ __forceinline__ void for_products(const int64_t *__restrict__ rpA, const int32_t *__restrict__ cA,
                                             const V *__restrict__ vA, const int64_t *__restrict__ rpB,
                                             const int32_t *__restrict__ cB, const V *__restrict__ vB,
                                             int64_t i, const int32_t *__restrict__ woff, int nwin, int w,
                                             int w_end, Chunk<BS, V> &L, F &&f,
                                             const uint2 *__restrict__ rB = nullptr) {
  const int t = threadIdx.x;
  const int64_t pa = rpA[i], pe = rpA[i + 1];
  for (int64_t p0 = pa; p0 < pe; p0 += BS) {
    const int cnt = (int)min((int64_t)BS, pe - p0);
    int32_t len = 0;
    int64_t st = 0;
    V a{};
    if (t < cnt) {
      const int32_t k = cA[p0 + t];
      st = rpB[k];
      if (woff) {
        const int32_t *wk = woff + (int64_t)k * (nwin + 1);
        const int32_t o0 = wk[w], o1 = wk[w_end];
        st += o0;
        len = o1 - o0;
      } else {
        len = (int32_t)(rpB[k + 1] - st);
      }
      if (VALS) a = vA[p0 + t];
    }
    const int32_t total = layout_chunk<BS, VALS, V>(len, st, a, L);
    walk_chunk<BS, U, VALS, V, PIPE, REC>(cB, vB, cnt, total, L, f, 0, rB);
    __syncthreads();
  }
}

// Rows of a bin are handed out from a global counter, `step` consecutive
// rows per fetch: thread 0 claims them and the block reads the first index
// back through LDS.  (One row per fetch left bins of millions of small rows
// bound by the throughput of atomics on that one counter.)  Callers fetch
// before their loop and again at the end of its body, and walk the claimed
// rows in an inner counted loop, so every loop test is on a block-uniform
// value and no thread-dependent branch leads into a loop header.  (With the
// fetch at the top of an endless loop, the compiler was free to route
// threads other than 0 from the end of the body straight past the fetch; the
// generated code then kept those lanes in an inner loop over the same row
// that they never left.)
__device__ __forceinline__ int64_t next_row(int64_t *ctr, int step = 1) {
  __shared__ int64_t r;
  if (threadIdx.x == 0) r = (int64_t)atomicAdd((unsigned long long *)ctr, (unsigned long long)step);
  __syncthreads();
  const int64_t v = r;
  __syncthreads();
  return v;
}

// Rows per fetch for a bin of `rows` rows on `grid` blocks: about 16
// fetches per block, 1 to 32 rows each.
inline int fetch_step(int64_t rows, int64_t grid) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(32, rows / std::max<int64_t>(1, grid * 16)));
}

template <int BS, class T> __device__ __forceinline__ T block_sum(T v, T *tmp) {
  T tot;
  block_excl_scan<BS>(v, tmp, &tot);
  return tot;
}

// ------------------------------------------------------------- symbolic --
template <int BS, int TBL>
__global__ void __launch_bounds__(BS) sym_hash(const int32_t *__restrict__ list, const int64_t *__restrict__ info,
                                               int bin, const int64_t *__restrict__ rpA,
                                               const int32_t *__restrict__ cA, const int64_t *__restrict__ rpB,
                                               const int32_t *__restrict__ cB, int64_t *__restrict__ nnz_row,
                                               int64_t *ctr, int step, int64_t *err) {
  constexpr int LG = __builtin_ctz(TBL);
  __shared__ int32_t keys[TBL];
  __shared__ Chunk<BS, uint8_t> L;
  __shared__ int64_t red[BS / WAVE + 1];
  const int64_t count = info[bin];
  const int32_t *rows = list + info[NBIN + bin];
  for (int64_t r0 = next_row(ctr, step); r0 < count; r0 = next_row(ctr, step)) {
   const int64_t r1 = min(r0 + (int64_t)step, count);
   for (int64_t r = r0; r < r1; r++) {
    const int64_t i = rows[r];
    for (int s = threadIdx.x; s < TBL; s += BS) keys[s] = EMPTY;
    __syncthreads();
    int64_t mine = 0;
    for_products<BS, false, uint8_t>(rpA, cA, (const uint8_t *)nullptr, rpB, cB, (const uint8_t *)nullptr, i,
                                     nullptr, 0, 0, 1, L, [&](int32_t j, uint8_t, uint8_t) {
      uint32_t h = hash_slot(j, LG);
      // the table is sized to at least twice the row's products; the probe
      // bound only guards against a broken invariant
      for (int probes = 0;; probes++) {
        if (probes >= TBL) { atomicAdd((unsigned long long *)err, 1ull); break; }
        const int32_t k = keys[h];
        if (k == j) break;
        if (k == EMPTY) {
          const int32_t old = atomicCAS(&keys[h], EMPTY, j);
          if (old == EMPTY) { mine++; break; }
          if (old == j) break;
        }
        h = (h + 1) & (TBL - 1);
      }
    });
    const int64_t tot = block_sum<BS>(mine, red);
    if (threadIdx.x == 0) nnz_row[i] = tot;
   }
  }
}

// bitmap over a window of `wbits` columns (dynamic LDS); rows wider than
// the window are walked once per window.
template <int BS>
__global__ void __launch_bounds__(BS) sym_bitmap(const int32_t *__restrict__ list, const int64_t *__restrict__ info,
                                                 int bin, const int64_t *__restrict__ rpA,
                                                 const int32_t *__restrict__ cA, const int64_t *__restrict__ rpB,
                                                 const int32_t *__restrict__ cB, int64_t ncols, int32_t wwords,
                                                 const int32_t *__restrict__ woff, int nwin,
                                                 int64_t *__restrict__ nnz_row, int64_t *ctr, int step) {
  extern __shared__ uint32_t bits[];
  __shared__ Chunk<BS, uint8_t> L;
  __shared__ int64_t red[BS / WAVE + 1];
  const int64_t count = info[bin];
  const int32_t *rows = list + info[NBIN + bin];
  const int64_t wcols = (int64_t)wwords * 32;
  for (int64_t r0 = next_row(ctr, step); r0 < count; r0 = next_row(ctr, step)) {
   const int64_t r1 = min(r0 + (int64_t)step, count);
   for (int64_t r = r0; r < r1; r++) {
    const int64_t i = rows[r];
    int64_t mine = 0;
    for (int64_t w0 = 0, wi = 0; w0 < ncols; w0 += wcols, wi++) {
      for (int s = threadIdx.x; s < wwords; s += BS) bits[s] = 0;
      __syncthreads();
      // with several windows, the window table limits each pass to its own
      // products (each product is walked once over all passes)
      // (two tiles in flight: the walk only gathers column indices)
      for_products<BS, false, uint8_t, SYM_U, true>(
          rpA, cA, (const uint8_t *)nullptr, rpB, cB, (const uint8_t *)nullptr, i, nwin > 1 ? woff : nullptr, nwin,
          (int)wi, (int)wi + 1, L, [&](int32_t j, uint8_t, uint8_t) {
        const int64_t jj = (int64_t)j - w0;
        if (jj >= 0 && jj < wcols) atomicOr(&bits[jj >> 5], 1u << (jj & 31));
      });
      for (int s = threadIdx.x; s < wwords; s += BS) mine += __popc(bits[s]);
      __syncthreads();
    }
    const int64_t tot = block_sum<BS>(mine, red);
    if (threadIdx.x == 0) nnz_row[i] = tot;
   }
  }
}

// -------------------------------------------------------------- numeric --
// Output bookkeeping: row_kept[i] = entries written; any_short is raised if
// some result equalled the identity and was dropped, or was written with
// column -1 (ranked groups of the dense windows), so that a compaction
// follows.

// EXTRACT: 0 = sorted (kept entries compacted, then bitonic-sorted by column), 2 = table order
template <class SR, int BS, int TBL, int EXTRACT>
__global__ void __launch_bounds__(BS) num_hash(const int32_t *__restrict__ list, const int64_t *__restrict__ info,
                                               int bin, const int64_t *__restrict__ rpA,
                                               const int32_t *__restrict__ cA,
                                               const typename SR::val_t *__restrict__ vA,
                                               const int64_t *__restrict__ rpB, const int32_t *__restrict__ cB,
                                               const typename SR::val_t *__restrict__ vB, int64_t ncols,
                                               int32_t wwords, OutRows orows,
                                               int32_t *__restrict__ cC, typename SR::val_t *__restrict__ vC,
                                               typename SR::acc_t id, int64_t *__restrict__ row_kept,
                                               int32_t *any_short, int64_t *ctr, int step) {
  using V = typename SR::val_t;
  using A = typename SR::acc_t;
  constexpr int LG = __builtin_ctz(TBL);
  constexpr int NV = SR::HAS_VALS ? TBL : 1;
  __shared__ int32_t keys[TBL];
  __shared__ A vals[NV];
  __shared__ Chunk<BS, V> L;
  __shared__ int64_t red[BS / WAVE + 1];
  const int64_t count = info[bin];
  const int32_t *rows = list + info[NBIN + bin];
  for (int64_t r0 = next_row(ctr, step); r0 < count; r0 = next_row(ctr, step)) {
   const int64_t r1 = min(r0 + (int64_t)step, count);
   for (int64_t r = r0; r < r1; r++) {
    const int64_t i = rows[r];
    for (int s = threadIdx.x; s < TBL; s += BS) {
      keys[s] = EMPTY;
      if (SR::HAS_VALS) vals[s] = id;
    }
    __syncthreads();
    for_products<BS, SR::HAS_VALS, V>(rpA, cA, vA, rpB, cB, vB, i, nullptr, 0, 0, 1, L, [&](int32_t j, V a, V b) {
      if (SR::HAS_VALS && (SR::absent(a, id) || SR::absent(b, id))) return;
      uint32_t h = hash_slot(j, LG);
      // the table holds at least twice the row's (symbolic) outputs
      bool placed = false;
      for (int probes = 0; probes < TBL; probes++) {
        const int32_t k = keys[h];
        if (k == j) { placed = true; break; }
        if (k == EMPTY) {
          const int32_t old = atomicCAS(&keys[h], EMPTY, j);
          if (old == EMPTY || old == j) { placed = true; break; }
        }
        h = (h + 1) & (TBL - 1);
      }
      if (!placed) { atomicOr(any_short + 1, 1); return; }
      if (SR::HAS_VALS) SR::lds_add(&vals[h], SR::mul(a, b));
    });
    __syncthreads();
    const int64_t base = orows.start[i];
    const int32_t coff = (int32_t)orows.col_off;
    int64_t written = 0;
    if (EXTRACT == 2) {
      // compact in table order (unsorted output)
      for (int c0 = 0; c0 < TBL; c0 += BS) {
        const int s = c0 + threadIdx.x;
        const int32_t kk = keys[s];
        const A v = SR::HAS_VALS ? vals[s] : (A)1;
        const int keep = (kk != EMPTY && !SR::acc_absent(v, id)) ? 1 : 0;
        int64_t tot;
        const int64_t pre = block_excl_scan<BS>((int64_t)keep, red, &tot);
        if (keep) {
          cC[base + written + pre] = kk + coff;
          vC[base + written + pre] = SR::out(v);
        }
        written += tot;
      }
    } else {
      // sorted output: gather the kept entries (results equal to the
      // identity are dropped) to the front of the table, bitonic-sort the
      // next power of two of them by column, write them out in order
      constexpr int PER = TBL / BS;
      int32_t kk[PER];
      A vv[PER];
      int32_t mine = 0;
#pragma unroll
      for (int q = 0; q < PER; q++) {
        const int s = q * BS + threadIdx.x;
        kk[q] = keys[s];
        vv[q] = SR::HAS_VALS ? vals[s] : (A)1;
        if (kk[q] != EMPTY && SR::acc_absent(vv[q], id)) kk[q] = EMPTY;
        mine += kk[q] != EMPTY ? 1 : 0;
      }
      int32_t cnt;
      int32_t pos = block_excl_scan<BS, int32_t>(mine, L.tmp, &cnt);  // ends with a barrier: table reads done
      // When B's columns fit a bitmap in the table's own LDS (with a word
      // prefix array beside it), the kept entries are placed by rank: mark
      // their columns, scan the popcounts once, and every entry's position
      // is the number of marked columns before it -- column order without
      // a sort (the table was read into registers above).
      const int nbw = (int)((ncols + 31) >> 5);
      const bool by_rank = SR::HAS_VALS ? (nbw <= TBL && nbw * 4 <= NV * (int)sizeof(A)) : (2 * nbw <= TBL);
      if (by_rank) {
        uint32_t *bm = reinterpret_cast<uint32_t *>(keys);
        uint32_t *pre = SR::HAS_VALS ? reinterpret_cast<uint32_t *>(vals) : bm + nbw;
        for (int u = threadIdx.x; u < nbw; u += BS) bm[u] = 0u;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; q++) {
          // a column outside B (a malformed operand) is dropped, never marked
          if (kk[q] != EMPTY && (uint32_t)kk[q] >= (uint32_t)ncols) kk[q] = EMPTY;
          if (kk[q] != EMPTY) atomicOr(&bm[kk[q] >> 5], 1u << (kk[q] & 31));
        }
        __syncthreads();
        const int per = (nbw + BS - 1) / BS;
        const int u0 = min((int)threadIdx.x * per, nbw), u1 = min(u0 + per, nbw);
        int32_t c = 0;
        for (int u = u0; u < u1; u++) c += __popc(bm[u]);
        int32_t tot;
        int32_t rk = block_excl_scan<BS, int32_t>(c, L.tmp, &tot);
        for (int u = u0; u < u1; u++) {
          pre[u] = (uint32_t)rk;
          rk += __popc(bm[u]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; q++) {
          if (kk[q] == EMPTY) continue;
          const int32_t j = kk[q];
          const int64_t o = base + (int64_t)pre[j >> 5] + __popc(bm[j >> 5] & ((1u << (j & 31)) - 1u));
          cC[o] = j + coff;
          vC[o] = SR::out(vv[q]);
        }
        written = cnt;
      } else {
#pragma unroll
      for (int q = 0; q < PER; q++) {
        if (kk[q] != EMPTY) {
          keys[pos] = kk[q];
          if (SR::HAS_VALS) vals[pos] = vv[q];
          pos++;
        }
      }
      const int P = cnt <= 1 ? 1 : 1 << (32 - __clz(cnt - 1));  // next power of two >= cnt
      // With column < 2^(32 - PB) for PB = log2(P) position bits, a kept
      // entry's column and compacted position pack into one 32-bit word;
      // sorting the words moves a third of the bytes of sorting (key,
      // value) pairs, and the values are read from their slots afterwards.
      const int PB = 31 - __clz(max(P, 2));
      const bool packed = SR::HAS_VALS && ncols <= ((int64_t)1 << (32 - PB));
      if (packed) {
        __syncthreads();  // the compacted entries come from other threads
        uint32_t *w32 = reinterpret_cast<uint32_t *>(keys);
        for (int s = threadIdx.x; s < P; s += BS)
          w32[s] = s < cnt ? ((uint32_t)keys[s] << PB) | (uint32_t)s : 0xffffffffu;
      } else {
        for (int s = cnt + threadIdx.x; s < P; s += BS) keys[s] = EMPTY;
      }
      __syncthreads();
      // While the stride is at most 64, the pairs of the 64 consecutive q
      // of one wave stay inside one 128-entry block that no other wave
      // touches, so consecutive passes with such strides need only a
      // wave-level sync; a block barrier separates the others.
      for (int k = 2; k <= P; k <<= 1) {
        for (int jst = k >> 1; jst > 0; jst >>= 1) {
          for (int q = threadIdx.x; q < P / 2; q += BS) {
            const int lo = q + (q & ~(jst - 1));  // jst is a power of two
            const int hi = lo + jst;
            const bool up = (lo & k) == 0;
            if (packed) {
              uint32_t *w32 = reinterpret_cast<uint32_t *>(keys);
              const uint32_t ka = w32[lo], kb = w32[hi];
              if ((ka > kb) == up) {
                w32[lo] = kb;
                w32[hi] = ka;
              }
            } else {
              const int32_t ka = keys[lo], kb = keys[hi];
              if ((ka > kb) == up) {
                keys[lo] = kb;
                keys[hi] = ka;
                if (SR::HAS_VALS) {
                  const A t = vals[lo];
                  vals[lo] = vals[hi];
                  vals[hi] = t;
                }
              }
            }
          }
          const int next = jst > 1 ? jst >> 1 : (2 * k <= P ? k : 0);
          if (jst > WAVE || next > WAVE || next == 0) {
            __syncthreads();
          } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          }
        }
      }
      if (packed) {
        const uint32_t *w32 = reinterpret_cast<const uint32_t *>(keys);
        const uint32_t pmask = (1u << PB) - 1u;
        for (int s = threadIdx.x; s < cnt; s += BS) {
          const uint32_t wv = w32[s];
          cC[base + s] = (int32_t)(wv >> PB) + coff;
          vC[base + s] = SR::out(vals[wv & pmask]);
        }
      } else {
        for (int s = threadIdx.x; s < cnt; s += BS) {
          cC[base + s] = keys[s] + coff;
          vC[base + s] = SR::out(SR::HAS_VALS ? vals[s] : (A)1);
        }
      }
      written = cnt;
      }
    }
    if (threadIdx.x == 0) {
      row_kept[i] = written;
      if (written != orows.count[i]) atomicOr(any_short, 1);
    }
    __syncthreads();
   }
  }
}

// Extraction of one dense window: `bits` marks the touched columns (for the
// boolean semiring they are the values), `vals` holds the accumulators of a
// value semiring.  Every touched slot is written out in column order, one
// holding the identity (an exact cancellation, a clamped sum) with column -1
// and *marked raised, so the compaction after the numeric pass drops it;
// touched slots and their bits are reset.  Ranks need only the bits'
// popcounts, not the accumulators.  Wave
// wv owns words [wv*WPW, (wv+1)*WPW); a lane takes one word, or a part of
// one (LPW lanes per word when a wave has more lanes than words, so no lane
// idles), and walks its set bits; ranks come from wave scans of the
// per-lane counts (adjacent lanes hold adjacent parts, so lane order is
// column order) and one block-level prefix over the waves.  Returns the
// number of entries written, marked ones included (the same on every
// thread).
template <class SR, int BS, int W>
__device__ __forceinline__ int64_t extract_window(typename SR::acc_t *vals, uint32_t *bits, typename SR::acc_t id,
                                                  int64_t w0, int64_t pos0, int32_t *__restrict__ cC,
                                                  typename SR::val_t *__restrict__ vC, int64_t *red,
                                                  int32_t *marked) {
  using A = typename SR::acc_t;
  constexpr bool VALS = SR::HAS_VALS;
  constexpr int NW = BS / WAVE, NWORD = W / 32, WPW = NWORD / NW;
  constexpr int LPW = WPW >= WAVE ? 1 : WAVE / WPW;  // lanes per word
  constexpr int BPL = 32 / LPW;                      // bits per lane
  constexpr uint32_t MASK = BPL == 32 ? 0xffffffffu : (1u << BPL) - 1u;
  constexpr int NG = (WPW * LPW + WAVE - 1) / WAVE;
  static_assert(NWORD % NW == 0 && 32 % LPW == 0, "window split");
  const int wv = threadIdx.x / WAVE, l = lane_id();
  // touched columns per lane part (popcounts, recomputed in the write pass)
  int64_t wtot = 0;
#pragma unroll 2
  for (int g = 0; g < NG; g++) {
    const int slot = g * WAVE + l;
    const int uw = slot / LPW, sh = (slot % LPW) * BPL;
    const int u = wv * WPW + uw;
    const uint32_t wd = uw < WPW ? (bits[u] >> sh) & MASK : 0u;
    wtot += wave_sum((int32_t)__popc(wd));
  }
  if (l == 0) red[wv] = wtot;
  __syncthreads();
  int64_t before = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < NW; q++) {
    const int64_t x = red[q];
    if (q < wv) before += x;
    tot += x;
  }
  int64_t pos = pos0 + before;
  bool any = false;
#pragma unroll 2
  for (int g = 0; g < NG; g++) {
    const int slot = g * WAVE + l;
    const int uw = slot / LPW, sh = (slot % LPW) * BPL;
    const int u = wv * WPW + uw;
    const int32_t c = uw < WPW ? __popc((bits[u] >> sh) & MASK) : 0;
    const int32_t inc = wave_incl_scan(c);
    int64_t p = pos + (inc - c);
    uint32_t wd = uw < WPW ? (bits[u] >> sh) & MASK : 0u;
    // every part of word u is read before part 0 clears it
    if constexpr (LPW > 1) __builtin_amdgcn_wave_barrier();
    if (uw < WPW && sh == 0) bits[u] = 0;
    while (wd) {
      const int b = __ffs(wd) - 1;
      wd &= wd - 1;
      const int s = u * 32 + sh + b;
      A v = (A)1;
      bool absent = false;
      if (VALS) {
        v = vals[s];
        vals[s] = id;
        absent = SR::acc_absent(v, id);
        any |= absent;
      }
      cC[p] = absent ? -1 : (int32_t)(w0 + s);
      vC[p] = SR::out(v);
      p++;
    }
    pos += lane63(inc);
  }
  if (any) atomicOr(marked, 1);
  __syncthreads();
  return tot;
}

// Ranked groups for sparse stretches of a dense row.  A run of consecutive
// windows whose products together fit one batch per thread (at most CAP) is
// handled in two passes over the same gathered products, held in registers:
// the first marks the touched columns in a bitmap over the run, a block scan
// of the bitmap's popcounts then ranks every touched column (its position in
// column order), and the second pass adds each product into a compact array
// at its column's rank.  The array is already in column order, so extraction
// writes it out as it stands.  The bitmap, the per-word rank prefixes, the
// columns and the accumulators share the LDS of the dense window; SPANW (the
// windows one run may cover) is what the bitmap and prefixes leave room for.
template <class SR, int BS, int W> struct RankWin {
  using A = typename SR::acc_t;
  static constexpr int RB = W * (int)sizeof(A);
  static constexpr int CAP = BS * WALK_U;
  static constexpr int WPW = W / 32;
  static constexpr int FIT = (RB - CAP * (4 + (int)sizeof(A))) / 8 / WPW;
  static constexpr int SPANW = FIT < 32 ? FIT : 32;
  static constexpr int NBW = SPANW * WPW;
  static constexpr bool OK = SR::HAS_VALS && SPANW >= 2;
  // byte offsets: accumulators, columns, bitmap, prefixes
  static constexpr int OFF_C = CAP * (int)sizeof(A);
  static constexpr int OFF_B = OFF_C + CAP * 4;
  static constexpr int OFF_P = OFF_B + NBW * 4;
  static_assert(!OK || OFF_P + NBW * 4 <= RB, "ranked group layout");
};
constexpr int NWPW = 256;  // most windows a row may split into for ranked groups

// Ranks of a marked run of nbw bitmap words: thread t takes a contiguous run
// of words, so one block scan of the per-thread popcounts gives every word's
// prefix; each touched column is listed at its rank with its accumulator
// reset.  Returns the number of touched columns (the same on every thread).
template <class SR, int BS>
__device__ __forceinline__ int32_t rank_run(const uint32_t *rbits, int32_t *rpre, int32_t *rcol,
                                            typename SR::acc_t *racc, int nbw, typename SR::acc_t id,
                                            int64_t *red) {
  const int per = (nbw + BS - 1) / BS;
  const int u0 = threadIdx.x * per, u1 = min(u0 + per, nbw);
  int64_t mine = 0;
  for (int u = u0; u < u1; u++) mine += __popc(rbits[u]);
  int64_t tot;
  int32_t r = (int32_t)block_excl_scan<BS, int64_t, false>(mine, red, &tot);
  for (int u = u0; u < u1; u++) {
    rpre[u] = r;
    uint32_t wd = rbits[u];
    while (wd) {
      const int b = __ffs(wd) - 1;
      wd &= wd - 1;
      rcol[r] = u * 32 + b;
      racc[r] = id;
      r++;
    }
  }
  return (int32_t)tot;
}

// Extraction of a ranked group: the n accumulators are in column order and
// each is written at its rank (thread t takes ranks t, t + BS, ..., so a
// wave's stores are contiguous), with no count and no scan.  An identity
// result (an exact cancellation, a clamped sum) is written with column -1
// and raises *marked; the compaction after the numeric pass drops such
// entries.  The bitmap is cleared.  Returns n.
template <class SR, int BS>
__device__ __forceinline__ int32_t extract_ranked(const typename SR::acc_t *racc, const int32_t *rcol,
                                                  uint32_t *rbits, int nbw, int n, typename SR::acc_t id,
                                                  int64_t col0, int64_t pos0, int32_t *__restrict__ cC,
                                                  typename SR::val_t *__restrict__ vC, int32_t *marked) {
  bool any = false;
  for (int r = threadIdx.x; r < n; r += BS) {
    const typename SR::acc_t v = racc[r];
    const bool absent = SR::acc_absent(v, id);
    any |= absent;
    cC[pos0 + r] = absent ? -1 : (int32_t)(col0 + rcol[r]);
    vC[pos0 + r] = SR::out(v);
  }
  if (any) atomicOr(marked, 1);
  for (int u = threadIdx.x; u < nbw; u += BS) rbits[u] = 0;
  __syncthreads();
  return n;
}

// Dense rows, window by window: W consecutive columns held in LDS as dense
// accumulators (values for value semirings, presence bits for the boolean
// one).  The window table gives, for every row k of B, where each window
// starts in B_k (B rows have ascending columns), so each product is visited
// exactly once over all windows.  A rows of at most BS entries keep their
// entries in registers across the windows and fetch the next group's table
// entries one group ahead; the next group's layout and first B loads are
// issued before the current one is written out, and inside a group each
// tile's loads are issued before the tile before it is consumed.  For value
// semirings, rows of at most BS A entries and moderate output counts first
// count their products per window (one pass over the A row's window-table
// entries): windows without products are skipped, and runs of sparse
// windows become ranked groups (above), so a row with few outputs spread
// over many windows pays for a few passes instead of one per window.
// Longer A rows are re-read in chunks for every window.  For 4-byte values
// B is read from rB, its entries as (column, value) records starting at
// position rowptr[0].
// At most 128 VGPRs (four waves per SIMD): two 512-thread blocks per CU when
// the LDS allows, one 1024-thread block otherwise (at 129 registers the
// fp64 instance lost half its blocks).
template <class SR, int BS, int W>
__global__ void __launch_bounds__(BS, 4) num_dense(const int32_t *__restrict__ list, const int64_t *__restrict__ info,
                                                int bin, const int64_t *__restrict__ rpA,
                                                const int32_t *__restrict__ cA,
                                                const typename SR::val_t *__restrict__ vA,
                                                const int64_t *__restrict__ rpB, const int32_t *__restrict__ cB,
                                                const typename SR::val_t *__restrict__ vB, int64_t ncols,
                                                const int32_t *__restrict__ woff, int nwin,
                                                OutRows orows, int32_t *__restrict__ cC,
                                                typename SR::val_t *__restrict__ vC, typename SR::acc_t id,
                                                int64_t *__restrict__ row_kept, int32_t *any_short,
                                                int64_t *ctr, int step, const uint2 *__restrict__ rB) {
  using V = typename SR::val_t;
  using A = typename SR::acc_t;
  using R = RankWin<SR, BS, W>;
  constexpr bool VALS = SR::HAS_VALS;
  constexpr bool REC = b_records<SR>();
  // records indexed by B position
  if constexpr (REC) rB -= rpB[0];
  constexpr int NWORD = W / 32;
  constexpr int NV = VALS ? W : 1;
  __shared__ __align__(16) A vals[NV];
  __shared__ uint32_t bits[NWORD];
  __shared__ Chunk<BS, V> L;
  __shared__ int64_t red[BS / WAVE + 1];
  __shared__ unsigned long long pw[R::OK ? NWPW : 1];
  // the ranked-group view of the accumulator space
  char *const region = reinterpret_cast<char *>(vals);
  A *const racc = reinterpret_cast<A *>(region);
  int32_t *const rcol = reinterpret_cast<int32_t *>(region + R::OFF_C);
  uint32_t *const rbits = reinterpret_cast<uint32_t *>(region + R::OFF_B);
  int32_t *const rpre = reinterpret_cast<int32_t *>(region + R::OFF_P);
  const int t = threadIdx.x;
  for (int s = t; s < NV; s += BS) vals[s] = id;
  for (int s = t; s < NWORD; s += BS) bits[s] = 0;
  __syncthreads();
  bool ranked_ready = false;  // the space holds a cleared ranked-group bitmap (else cleared dense accumulators)
  const bool can_rank = R::OK && woff != nullptr && nwin > 1 && nwin <= NWPW;
  const int64_t count = info[bin];
  const int32_t *rows = list + info[NBIN + bin];
  for (int64_t r0 = next_row(ctr, step); r0 < count; r0 = next_row(ctr, step)) {
   const int64_t r1 = min(r0 + (int64_t)step, count);
   for (int64_t r = r0; r < r1; r++) {
    const int64_t i = rows[r];
    const int64_t base = orows.start[i];
    const int64_t pa = rpA[i], pe = rpA[i + 1];
    int64_t written = 0;
    // rows with more than CAP/2 outputs per window on average stay dense
    const bool use_rank = can_rank && pe - pa <= BS && orows.count[i] <= (int64_t)nwin * (R::CAP / 2);
    if (use_rank) {
      for (int s = t; s < nwin; s += BS) pw[s] = 0;
      __syncthreads();
      // products per window: one (A entry, window) pair per thread, four at a time
      const int np = (int)(pe - pa) * nwin;
      for (int x0 = t; x0 < np; x0 += 4 * BS) {
        int32_t d[4];
        int sw[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int x = x0 + u * BS;
          d[u] = 0;
          sw[u] = 0;
          if (x < np) {
            const int e = x / nwin;
            sw[u] = x - e * nwin;
            const int32_t *wk = woff + (int64_t)cA[pa + e] * (nwin + 1) + sw[u];
            d[u] = wk[1] - wk[0];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
          if (d[u]) atomicAdd(&pw[sw[u]], (unsigned long long)d[u]);
      }
      __syncthreads();
    }
    // The group from window wa on: [ga, gb), dense or ranked (the same on
    // every thread).  Windows without products are skipped; a window with
    // more than CAP products is dense.  ga == nwin: no group left.
    auto next_group = [&](int wa, int &ga, int &gb) -> bool {
      if (!use_rank) {
        ga = wa;
        gb = wa + 1;
        return true;
      }
      while (wa < nwin && pw[wa] == 0) wa++;
      ga = wa;
      gb = wa + 1;
      if (wa >= nwin || pw[wa] > (unsigned long long)R::CAP) return true;
      unsigned long long sum = pw[wa];
      while (gb < nwin && gb - wa < R::SPANW && sum + pw[gb] <= (unsigned long long)R::CAP) sum += pw[gb++];
      return false;
    };
    // the accumulator space in the form the next group needs
    auto ready = [&](bool dense) {
      if (!R::OK || dense != ranked_ready) return;
      if (dense) {
        for (int s = t; s < NV; s += BS) vals[s] = id;
      } else {
        for (int s = t; s < R::NBW; s += BS) rbits[s] = 0;
      }
      __syncthreads();
      ranked_ready = !dense;
    };
    auto dense_add = [&](int64_t w0) {
      return [&, w0](int32_t j, V a, V b) {
        if (VALS && (SR::absent(a, id) || SR::absent(b, id))) return;
        const uint32_t jj = (uint32_t)j - (uint32_t)w0;
        if (jj >= (uint32_t)W) return;  // B rows must list columns in ascending order
        if constexpr (VALS) SR::lds_add(&vals[jj], SR::mul(a, b));
        atomicOr(&bits[jj >> 5], 1u << (jj & 31));
      };
    };
    // ranked groups: mark, then add at the column's rank
    auto rank_mark = [&](int64_t c0, int64_t span) {
      return [&, c0, span](int32_t j, V a, V b) {
        if constexpr (R::OK) {
          if (SR::absent(a, id) || SR::absent(b, id)) return;
          const uint32_t jl = (uint32_t)j - (uint32_t)c0;
          if (jl >= (uint32_t)span) return;
          atomicOr(&rbits[jl >> 5], 1u << (jl & 31));
        }
      };
    };
    auto rank_add = [&](int64_t c0, int64_t span) {
      return [&, c0, span](int32_t j, V a, V b) {
        if constexpr (R::OK) {
          if (SR::absent(a, id) || SR::absent(b, id)) return;
          const uint32_t c = (uint32_t)j - (uint32_t)c0;
          if (c >= (uint32_t)span) return;
          const int q = rpre[c >> 5] + __popc(rbits[c >> 5] & ((1u << (c & 31)) - 1u));
          SR::lds_add(&racc[q], SR::mul(a, b));
        }
      };
    };
    int ga, gb;
    bool dense = next_group(0, ga, gb);
    if (pe - pa <= BS) {
      // Group pipeline: while group g is written out, the layout of group
      // g+1 is already done and its first batch of B loads is in flight.
      // Skipped windows hold no products of the row, so every A entry's
      // table offset at the start of a group equals the one at the end of
      // the group before.  A ranked group's products fit the first batch.
      const int cnt = (int)(pe - pa);
      int32_t k = 0, o_cur = 0, o_nxt = 0;
      int64_t rb = 0;
      V av{};
      const int32_t *wk = nullptr;
      if (t < cnt) {
        k = cA[pa + t];
        rb = rpB[k];
        if (VALS) av = vA[pa + t];
        if (nwin > 1) {
          wk = woff + (int64_t)k * (nwin + 1);
          if (ga < nwin) {
            o_cur = wk[ga];
            o_nxt = wk[gb];
          }
        } else {
          o_nxt = (int32_t)(rpB[k + 1] - rb);
        }
      }
      int32_t total = layout_chunk<BS, VALS, V>(o_nxt - o_cur, rb + o_cur, av, L);
      Batch<WALK_U, V> g;
      gather_batch<BS, WALK_U, VALS, V, REC>(cB, vB, cnt, total, L, 0, g, rB);
      while (ga < nwin) {
        int na = nwin, nb = nwin;
        bool ndense = true;
        if (gb < nwin) ndense = next_group(gb, na, nb);
        const int32_t o_after = (wk && na < nwin) ? wk[nb] : 0;
        ready(dense);
        const int64_t c0 = (int64_t)ga * W;
        int32_t nrank = 0;
        if (dense || !R::OK) {
          // g holds the first tile; each further tile is gathered before
          // the one before it is consumed
          for (int32_t b0 = 0; b0 < total; b0 += BS * WALK_U) {
            Batch<WALK_U, V> h = g;
            if (b0 + BS * WALK_U < total)
              gather_batch<BS, WALK_U, VALS, V, REC>(cB, vB, cnt, total, L, b0 + BS * WALK_U, h, rB);
            consume_batch<BS, WALK_U, V>(g, L, b0, total, dense_add(c0));
            g = h;
          }
        } else {
          const int64_t span = (int64_t)(gb - ga) * W;
          consume_batch<BS, WALK_U, V>(g, L, 0, total, rank_mark(c0, span));
          __syncthreads();
          nrank = rank_run<SR, BS>(rbits, rpre, rcol, racc, (gb - ga) * R::WPW, id, red);
          __syncthreads();
          consume_batch<BS, WALK_U, V>(g, L, 0, total, rank_add(c0, span));
        }
        __syncthreads();  // group accumulated; L free
        int32_t total_n = 0;
        if (na < nwin) {
          total_n = layout_chunk<BS, VALS, V>(o_after - o_nxt, rb + o_nxt, av, L);
          gather_batch<BS, WALK_U, VALS, V, REC>(cB, vB, cnt, total_n, L, 0, g, rB);
        }
        if (dense || !R::OK)
          written += extract_window<SR, BS, W>(vals, bits, id, c0 + orows.col_off, base + written, cC, vC, red, any_short);
        else
          written += extract_ranked<SR, BS>(racc, rcol, rbits, (gb - ga) * R::WPW, nrank, id, c0 + orows.col_off,
                                            base + written, cC, vC, any_short);
        total = total_n;
        o_nxt = o_after;
        ga = na;
        gb = nb;
        dense = ndense;
      }
    } else {
      ready(true);
      for (int w = 0; w < nwin; w++) {
        const int64_t w0 = (int64_t)w * W;
        for_products<BS, VALS, V, WALK_U, true, REC>(rpA, cA, vA, rpB, cB, vB, i, nwin > 1 ? woff : nullptr, nwin,
                                                     w, w + 1, L, dense_add(w0), rB);
        written += extract_window<SR, BS, W>(vals, bits, id, w0 + orows.col_off, base + written, cC, vC, red, any_short);
      }
    }
    if (t == 0) {
      row_kept[i] = written;
      if (written != orows.count[i]) atomicOr(any_short, 1);
    }
   }
  }
}

// --------------------------------------------------------------- masked --
// C = M (.) (A (x) B): only positions in M's pattern are formed (an output
// with predefined sparsity, Sections 1 and 7).  The work items are (row,
// chunk of LM consecutive mask entries of the row), handed out heaviest
// first from one counter, so the chunks of a long mask row run on several
// blocks at once instead of one after another on one.  A block stages its
// chunk's sorted columns in LDS with their accumulators beside them, every
// product of the row finds its column by binary search among them (products
// outside the chunk are dropped), and the kept entries are written in mask
// order into the chunk's own mask-aligned segment; kept[x] counts them for
// the final compaction.
template <class SR, int BS>
__device__ __forceinline__ int64_t write_kept(const typename SR::acc_t *vals, const int32_t *keys, int n,
                                              typename SR::acc_t id, int64_t pos0, int32_t *__restrict__ cC,
                                              typename SR::val_t *__restrict__ vC, int64_t *red) {
  constexpr int NW = BS / WAVE;
  const int wv = threadIdx.x / WAVE, l = lane_id();
  const int span = ((n + NW * WAVE - 1) / (NW * WAVE)) * WAVE;  // slots per wave, whole waves
  const int b0 = wv * span, b1 = min(b0 + span, n);
  int64_t cnt = 0;
  for (int g = b0; g < b0 + span; g += WAVE) {
    const int q = g + l;
    cnt += __popcll(__ballot(q < b1 && !SR::acc_absent(vals[q], id)));
  }
  if (l == 0) red[wv] = cnt;
  __syncthreads();
  int64_t before = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < NW; q++) {
    const int64_t x = red[q];
    if (q < wv) before += x;
    tot += x;
  }
  int64_t pos = pos0 + before;
  const uint64_t lt = lanemask_lt();
  for (int g = b0; g < b0 + span; g += WAVE) {
    const int q = g + l;
    const typename SR::acc_t v = q < b1 ? vals[q] : id;
    const bool keep = q < b1 && !SR::acc_absent(v, id);
    const uint64_t mk = __ballot(keep);
    if (keep) {
      const int64_t o = pos + __popcll(mk & lt);
      cC[o] = keys[q];
      vC[o] = SR::out(v);
    }
    pos += __popcll(mk);
  }
  __syncthreads();
  return tot;
}

template <class SR, int BS, int LM>
__global__ void __launch_bounds__(BS) masked_rows(const int64_t *__restrict__ rpA, const int32_t *__restrict__ cA,
                                                  const typename SR::val_t *__restrict__ vA,
                                                  const int64_t *__restrict__ rpB, const int32_t *__restrict__ cB,
                                                  const typename SR::val_t *__restrict__ vB,
                                                  const int64_t *__restrict__ rpM, const int32_t *__restrict__ cM,
                                                  const int32_t *__restrict__ irow,
                                                  const int32_t *__restrict__ ichunk,
                                                  const int32_t *__restrict__ order, int64_t items,
                                                  int32_t *__restrict__ cC, typename SR::val_t *__restrict__ vC,
                                                  typename SR::acc_t id, int64_t *__restrict__ kept, int64_t *ctr) {
  using V = typename SR::val_t;
  using A = typename SR::acc_t;
  __shared__ int32_t keys[LM];
  __shared__ A vals[LM];
  __shared__ Chunk<BS, V> L;
  __shared__ int64_t red[BS / WAVE + 1];
  const int t = threadIdx.x;
  for (int64_t r = next_row(ctr); r < items; r = next_row(ctr)) {
    const int32_t x = order[r];
    const int64_t i = irow[x];
    const int64_t s0 = rpM[i] + (int64_t)ichunk[x] * LM;
    const int n = (int)min((int64_t)LM, rpM[i + 1] - s0);
    for (int q = t; q < n; q += BS) {
      keys[q] = cM[s0 + q];
      vals[q] = id;
    }
    __syncthreads();
    const int32_t c_lo = keys[0], c_hi = keys[n - 1];
    for_products<BS, SR::HAS_VALS, V>(rpA, cA, vA, rpB, cB, vB, i, nullptr, 0, 0, 1, L, [&](int32_t j, V a, V b) {
      if (SR::HAS_VALS && (SR::absent(a, id) || SR::absent(b, id))) return;
      if (j < c_lo || j > c_hi) return;
      int lo = 0, hi = n - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (keys[mid] < j) lo = mid + 1; else hi = mid;
      }
      if (keys[lo] != j) return;
      SR::lds_add(&vals[lo], SR::HAS_VALS ? SR::mul(a, b) : (A)1);
    });
    const int64_t written = write_kept<SR, BS>(vals, keys, n, id, s0, cC, vC, red);
    if (t == 0) kept[x] = written;
  }
}

// Masked work items per row: chunks of LM mask entries (none when the mask
// row or the A row is empty).
__global__ void masked_count_items(const int64_t *__restrict__ rpA, const int64_t *__restrict__ rpM, int64_t m,
                                   int lm, int64_t *__restrict__ cnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t nm = rpM[i + 1] - rpM[i];
    cnt[i] = (nm > 0 && rpA[i + 1] > rpA[i]) ? (nm + lm - 1) / lm : 0;
  }
}

// Item x of row i (items of a row are consecutive, from ioff[i]): its row,
// chunk, first mask position, weight (the row's products) and its slot in
// the launch order (identity; sorted heaviest first afterwards).
__global__ void masked_fill_items(const int64_t *__restrict__ ioff, const int64_t *__restrict__ rpM,
                                  const int64_t *__restrict__ w, int64_t m, int lm, int32_t *__restrict__ irow,
                                  int32_t *__restrict__ ichunk, int32_t *__restrict__ order,
                                  int64_t *__restrict__ witem, int64_t *__restrict__ src) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t x = ioff[i]; x < ioff[i + 1]; x++) {
      const int32_t c = (int32_t)(x - ioff[i]);
      irow[x] = (int32_t)i;
      ichunk[x] = c;
      order[x] = (int32_t)x;
      witem[x] = w[i];
      src[x] = rpM[i] + (int64_t)c * lm;
    }
  }
}

// C's row pointers from the items' output offsets: row i starts at its first
// item's offset (ioff[m] = number of items, koff[items] = nnz).
__global__ void masked_rowptr(const int64_t *__restrict__ ioff, const int64_t *__restrict__ koff, int64_t m,
                              int64_t *__restrict__ rp) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= m; i += (int64_t)gridDim.x * blockDim.x)
    rp[i] = koff[ioff[i]];
}

// Window table: woff[k*(nwin+1) + w] = first position in B_k with column
// >= w*W (relative to rowptr[k]); woff[k*(nwin+1)+nwin] = nnz(B_k).
__global__ void build_woff(const int64_t *__restrict__ rpB, const int32_t *__restrict__ cB, int64_t nrows,
                           int nwin, int64_t W, int32_t *__restrict__ woff) {
  const int64_t total = nrows * (nwin + 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / (nwin + 1);
    const int w = (int)(t % (nwin + 1));
    const int64_t a = rpB[k], b = rpB[k + 1];
    int64_t res;
    if (w == nwin) res = b - a;
    else {
      const int64_t target = (int64_t)w * W;
      int64_t lo = a, hi = b;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cB[mid] < target) lo = mid + 1; else hi = mid;
      }
      res = lo - a;
    }
    woff[t] = (int32_t)res;
  }
}

// Compaction after a numeric pass.  Row i of C was written as Q segments
// (segment q from start[q m + i], len[q m + i] entries; one segment per row
// outside the column-block path) that may fall short of the row's symbolic
// count (identity results dropped by the hash bins) and may hold entries
// with column -1 (identity results of dense windows and ranked groups,
// written in place).  The listed rows
// (rows = null: rows 0..n-1) are counted, then packed: cnt[i] = entries of
// row i with a column >= 0; they move in order to rp_new[i] onwards.  One
// wave per row.
__global__ void count_valid(const int32_t *__restrict__ rows, int64_t n, int Q, int64_t m,
                            const int64_t *__restrict__ start, const int64_t *__restrict__ len,
                            const int32_t *__restrict__ col, int64_t *__restrict__ cnt) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t r = wid; r < n; r += nw) {
    const int64_t i = rows ? rows[r] : r;
    int64_t acc = 0;
    for (int q = 0; q < Q; q++) {
      const int64_t a = start[(int64_t)q * m + i], e = a + len[(int64_t)q * m + i];
      for (int64_t t = a + lane_id(); t < e; t += WAVE) acc += col[t] >= 0 ? 1 : 0;
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) cnt[i] = acc;
  }
}

template <class V>
__global__ void compact_valid(const int32_t *__restrict__ rows, int64_t n, int Q, int64_t m,
                              const int64_t *__restrict__ start, const int64_t *__restrict__ len,
                              const int64_t *__restrict__ rp_new, const int32_t *__restrict__ c_old,
                              const V *__restrict__ v_old, int32_t *__restrict__ c_new, V *__restrict__ v_new) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  const uint64_t lt = lanemask_lt();
  for (int64_t r = wid; r < n; r += nw) {
    const int64_t i = rows ? rows[r] : r;
    int64_t o = rp_new[i];
    for (int q = 0; q < Q; q++) {
      const int64_t a = start[(int64_t)q * m + i], e = a + len[(int64_t)q * m + i];
      for (int64_t t0 = a; t0 < e; t0 += WAVE) {
        const int64_t t = t0 + lane_id();
        const int32_t c = t < e ? c_old[t] : -1;
        const uint64_t mk = __ballot(c >= 0);
        if (c >= 0) {
          const int64_t d = o + __popcll(mk & lt);
          c_new[d] = c;
          v_new[d] = v_old[t];
        }
        o += __popcll(mk);
      }
    }
  }
}

// Pack rows whose kept count fell short of a known count (the masked
// contraction's items).
template <class V>
__global__ void compact_rows(const int64_t *rp_old, const int64_t *rp_new, int64_t m, const int32_t *c_old,
                             const V *v_old, int32_t *c_new, V *v_new) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t i = wid; i < m; i += nw) {
    const int64_t a = rp_old[i], n = rp_new[i + 1] - rp_new[i], o = rp_new[i];
    for (int64_t q = lane_id(); q < n; q += WAVE) {
      c_new[o + q] = c_old[a + q];
      v_new[o + q] = v_old[a + q];
    }
  }
}

inline unsigned gridn(int64_t n, int bs = 256, int64_t cap = 65536) {
  int64_t g = (n + bs - 1) / bs;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Order the rows of one bin heaviest first (by their product counts), so the
// longest rows of a persistent launch start early instead of forming its tail.
void heavy_first(Ctx *c, int32_t *seg, int64_t nb, const int64_t *w, hipStream_t s) {
  if (nb < 2) return;
  Buf keys(c, sizeof(int64_t) * (size_t)nb);
  heavy_first_keys<<<gridn(nb), 256, 0, s>>>(seg, w, nb, keys.as<int64_t>());
  SRTC_LAUNCH_CHECK("heavy_first_keys");
  radix_sort_pairs(c, keys.as<int64_t>(), reinterpret_cast<uint32_t *>(seg), nb, 16, s);
}

// A table built from B alone for `key` (a window width, or -1 for the value
// records), `bytes` long: taken from the context when it keeps this B's
// tables (the row panels of one product), built there the first time;
// otherwise built into `local`.  build(dst) launches the kernels that fill
// it.
template <class Build>
const void *b_table(Ctx *c, const CsrView &Bm, int64_t key, size_t bytes, Buf &local, Build &&build) {
  const Ctx::KeptB &k = c->keep_b;
  const bool kept = k.rowptr && k.rowptr == Bm.rowptr && k.col == Bm.col && k.val == Bm.val && k.m == Bm.m &&
                    k.n == Bm.n && k.nnz == Bm.nnz;
  if (!kept) {
    local = Buf(c, bytes);
    build(local.p);
    return local.p;
  }
  for (const Ctx::BTable &t : c->b_tables)
    if (t.key == key) return t.buf.p;
  c->b_tables.push_back(Ctx::BTable{key, Buf(c, bytes)});
  void *p = c->b_tables.back().buf.p;
  build(p);
  return p;
}

// Schedules: symbolic hash ceiling, numeric bin edges, extraction and dense
// window shape.  Index = schedule id.
const Schedule kSchedules[SRTC_NUM_SCHEDULES] = {
    // sym_hash_max, t_tiny, t_small, t_mid, t_big, small_wave, dense_bs, dense_wide
    {2048, 32, 256, 2048, 4096, 0, 256, 0},   // 0 balanced
    {2048, 32, 256, 2048, 4096, 1, 256, 0},   // 1 as 0 with one wave per row in the 512-slot bin
    {2048, 32, 256, 256, 256, 1, 256, 0},     // 2 dense windows from 257 outputs
    {8192, 32, 256, 2048, 2048, 0, 1024, 1},  // 3 wide dense windows (1024-thread blocks) from 2049 outputs
    {0, 0, 0, 0, 0, 0, 256, 0},               // 4 dense windows for every row
    {2048, 32, 256, 256, 256, 0, 512, 0},     // 5 as 0, 512-thread dense windows from 257 outputs
    {2048, 32, 256, 2048, 4096, 0, 512, 2},   // 6 as 5 with narrow dense windows (more blocks per CU)
    {256, 32, 256, 1024, 1024, 1, 256, 0},    // 7 bitmap symbolic above 256 products
};

struct Launch {
  Ctx *c;
  hipStream_t s;
  int blocks_per_cu(int lds_bytes, int bs) const {
    int by_lds = lds_bytes > 0 ? LDS_BYTES / lds_bytes : 64;
    int by_waves = 32 / std::max(1, bs / WAVE);  // 8 waves/SIMD x 4 SIMDs
    return std::max(1, std::min(by_lds, by_waves));
  }
  unsigned grid(int64_t rows, int lds_bytes, int bs) const {
    int64_t cap = (int64_t)c->num_cus * blocks_per_cu(lds_bytes, bs);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(rows, cap));
  }
};

template <int BS, int TBL>
void launch_sym_hash(const Launch &L, int64_t rows, const int32_t *list, const int64_t *info, int bin,
                     const CsrView &A, const CsrView &B, int64_t *nnz_row, int64_t *ctr, int64_t *err) {
  if (rows == 0) return;
  const int lds = TBL * 4 + sizeof(Chunk<BS, uint8_t>) + 64;
  const unsigned grid = L.grid(rows, lds, BS);
  sym_hash<BS, TBL><<<grid, BS, 0, L.s>>>(list, info, bin, A.rowptr, A.col, B.rowptr, B.col, nnz_row, ctr,
                                          fetch_step(rows, grid), err);
  SRTC_LAUNCH_CHECK("sym_hash");
}

int32_t bitmap_words(int64_t ncols, int bs, int64_t budget_bytes) {
  int64_t want = (ncols + 31) / 32;
  int64_t cap = budget_bytes / 4;
  cap -= cap % bs;
  if (cap < bs) cap = bs;
  int64_t wv = std::min(want, cap);
  wv = ((wv + bs - 1) / bs) * bs;  // whole words per thread
  return (int32_t)wv;
}

// Symbolic pass over `nsel` rows (row ids in row_map, or 0..nsel-1) whose
// product counts are w (indexed by row id): nnz_row[row] for each.  Returns
// the product total.  Synchronizes once (bin sizes).
int64_t run_symbolic(const Launch &L, const Schedule &S, const CsrView &Am, const CsrView &Bm, const int64_t *w,
                     const int32_t *row_map, int64_t nsel, int64_t *info1, int32_t *list, int64_t *nnz_row,
                     int64_t *err) {
  hipStream_t s = L.s;
  Ctx *c = L.c;
  const int64_t n = Bm.n;
  // product counts in selection order
  Buf wbuf;
  const int64_t *wsel = w;
  if (row_map) {
    wbuf = Buf(c, sizeof(int64_t) * (size_t)std::max<int64_t>(nsel, 1));
    gather_i64<<<gridn(nsel), 256, 0, s>>>(w, row_map, nsel, wbuf.as<int64_t>());
    SRTC_LAUNCH_CHECK("gather_i64");
    wsel = wbuf.as<int64_t>();
  }
  Thresholds th1{};
  {
    // bins: 1: <=32 (64-slot hash), 2: <=256 (512), 3: <=2048 (4096),
    // 4: <=8192 (16384), 5: bitmap.  Edges above sym_hash_max collapse so
    // those rows fall through to the bitmap.
    const int64_t edges[4] = {32, 256, 2048, 8192};
    int64_t prev = 0;
    for (int b = 0; b < 4; b++) {
      th1.t[b] = edges[b] <= S.sym_hash_max ? edges[b] : prev;
      prev = th1.t[b];
    }
  }
  bin_count<<<gridn(nsel, 256, 2048), 256, 0, s>>>(wsel, nsel, th1, info1, Am.rowptr, row_map);
  SRTC_LAUNCH_CHECK("bin_count");
  bin_offsets<<<1, 64, 0, s>>>(info1);
  bin_scatter<<<gridn(nsel, 256, 4096), 256, 0, s>>>(wsel, nsel, th1, info1, list, row_map);
  SRTC_LAUNCH_CHECK("bin_scatter");
  int64_t hinfo[INFO];
  read_to_host(c, hinfo, info1, sizeof(hinfo), s);
  heavy_first(c, list + hinfo[NBIN + 5], hinfo[5], w, s);
  int64_t *ctr1 = info1 + 3 * NBIN;
  // algorithmic bytes of a symbolic bin: its A rows (pointers + columns),
  // B's columns once, one count per row
  auto sym_bytes = [&](int b) {
    return 16.0 * hinfo[b] + 4.0 * hinfo[SUMA + b] + 4.0 * Bm.nnz + 8.0 * (Bm.m + 1) + 8.0 * hinfo[b];
  };
  static const char *kSymName[NBIN] = {"", "spgemm.symbolic.hash64", "spgemm.symbolic.hash512",
                                       "spgemm.symbolic.hash4096", "spgemm.symbolic.hash16384",
                                       "spgemm.symbolic.bitmap"};
  for (int b = 1; b < NBIN - 1; b++) {
    if (hinfo[b] == 0) continue;
    ProfScope ps(c, kSymName[b], sym_bytes(b), s);
    if (b == 1) launch_sym_hash<64, 64>(L, hinfo[1], list, info1, 1, Am, Bm, nnz_row, ctr1 + 1, err);
    if (b == 2) launch_sym_hash<64, 512>(L, hinfo[2], list, info1, 2, Am, Bm, nnz_row, ctr1 + 2, err);
    if (b == 3) launch_sym_hash<256, 4096>(L, hinfo[3], list, info1, 3, Am, Bm, nnz_row, ctr1 + 3, err);
    if (b == 4) launch_sym_hash<512, 16384>(L, hinfo[4], list, info1, 4, Am, Bm, nnz_row, ctr1 + 4, err);
  }
  if (hinfo[5] > 0) {
    ProfScope ps(c, kSymName[5], sym_bytes(5), s);
    // 512 threads: the bitmap bounds blocks per CU, so larger blocks keep
    // more gathers in flight (R-MAT 18 squared: 7.8 -> 6.1 ms)
    constexpr int BS = 512;
    const int stat = (int)sizeof(Chunk<BS, uint8_t>) + 64;
    // at most 64 KB of bitmap (2^19 columns) per pass: two blocks per CU
    // instead of one; with the window table the extra passes only re-lay
    // the A row (R-MAT 21 panel squared, fp32: 213 -> 177 ms per product)
    const int32_t ww = bitmap_words(n, BS, std::min<int64_t>(std::min<int64_t>(LDS_BYTES, c->lds_budget) - stat - 1024,
                                                             64 * 1024));
    const int64_t wcols = (int64_t)ww * 32;
    const int nwin = (int)((n + wcols - 1) / wcols);
    Buf woff;
    const int32_t *wo = nullptr;
    if (nwin > 1)
      wo = (const int32_t *)b_table(L.c, Bm, wcols, sizeof(int32_t) * (size_t)(Bm.m * (nwin + 1)), woff, [&](void *d) {
        build_woff<<<gridn(Bm.m * (nwin + 1)), 256, 0, s>>>(Bm.rowptr, Bm.col, Bm.m, nwin, wcols, (int32_t *)d);
        SRTC_LAUNCH_CHECK("build_woff");
      });
    auto kern = sym_bitmap<BS>;
    if (ww * 4 > 64 * 1024)
      SRTC_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, ww * 4));
    kern<<<L.grid(hinfo[5], stat + ww * 4, BS), BS, (size_t)ww * 4, s>>>(list, info1, 5, Am.rowptr, Am.col,
                                                                      Bm.rowptr, Bm.col, n, ww, wo,
                                                                      nwin, nnz_row, ctr1 + 5, 1);
    SRTC_LAUNCH_CHECK("sym_bitmap");
  }
  return hinfo[4 * NBIN];
}

template <class SR> struct NumLaunch {
  using V = typename SR::val_t;
  using A = typename SR::acc_t;
  template <int BS, int TBL, int EX>
  static void hash(const Launch &L, int64_t rows, const int32_t *list, const int64_t *info, int bin,
                   const CsrView &Am, const CsrView &Bm, OutRows orows, int32_t *cC, V *vC, A id,
                   int64_t *kept, int32_t *any_short, int64_t *ctr) {
    if (rows == 0) return;
    constexpr int NV = SR::HAS_VALS ? TBL : 1;
    const int stat = TBL * 4 + NV * (int)sizeof(A) + (int)sizeof(Chunk<BS, V>) + 64;
    const unsigned grid = L.grid(rows, stat, BS);
    num_hash<SR, BS, TBL, EX><<<grid, BS, 0, L.s>>>(
        list, info, bin, Am.rowptr, Am.col, (const V *)Am.val, Bm.rowptr, Bm.col, (const V *)Bm.val, Bm.n, 0,
        orows, cC, vC, id, kept, any_short, ctr, fetch_step(rows, grid));
    SRTC_LAUNCH_CHECK("num_hash");
  }
  template <int BS, int W>
  static void dense(const Launch &L, int64_t rows, const int32_t *list, const int64_t *info, int bin,
                    const CsrView &Am, const CsrView &Bm, const int32_t *woff, int nwin, const uint2 *rB,
                    OutRows orows, int32_t *cC, V *vC, A id, int64_t *kept, int32_t *any_short, int64_t *ctr) {
    if (rows == 0) return;
    constexpr int NV = SR::HAS_VALS ? W : 1;
    const int stat = NV * (int)sizeof(A) + W / 8 + (int)sizeof(Chunk<BS, V>) + (RankWin<SR, BS, W>::OK ? NWPW * 8 : 8) + 64;
    num_dense<SR, BS, W><<<L.grid(rows, stat, BS), BS, 0, L.s>>>(
        list, info, bin, Am.rowptr, Am.col, (const V *)Am.val, Bm.rowptr, Bm.col, (const V *)Bm.val, Bm.n, woff,
        nwin, orows, cC, vC, id, kept, any_short, ctr, 1, rB);
    SRTC_LAUNCH_CHECK("num_dense");
  }
};

// Dense window width (columns) for a semiring and a schedule's width code
// (0: 64 KB of accumulators, 1: 128 KB, 2: 32 KB).
template <class SR> constexpr int64_t dense_width(int code) {
  if (!SR::HAS_VALS) return code == 1 ? (1 << 20) : code == 2 ? (1 << 17) : (1 << 18);
  return (code == 1 ? 16384 : code == 2 ? 4096 : 8192) * (8 / (int64_t)sizeof(typename SR::acc_t));
}

// LDS a block of each kernel uses (the same expressions as the launchers).
template <int BS> constexpr int sym_hash_lds(int tbl) { return tbl * 4 + (int)sizeof(Chunk<BS, uint8_t>) + 64; }
template <class SR, int BS> constexpr int num_hash_lds(int tbl) {
  return tbl * 4 + (SR::HAS_VALS ? tbl : 1) * (int)sizeof(typename SR::acc_t) +
         (int)sizeof(Chunk<BS, typename SR::val_t>) + 64;
}
template <class SR, int BS, int W> constexpr int num_dense_lds() {
  return (SR::HAS_VALS ? W : 1) * (int)sizeof(typename SR::acc_t) + W / 8 +
         (int)sizeof(Chunk<BS, typename SR::val_t>) + (RankWin<SR, BS, W>::OK ? NWPW * 8 : 8) + 64;
}

// A schedule as run under the context's LDS budget (SRTC_LDS_BUDGET): a
// hash bin whose kernel would need more LDS per block is merged into the
// next larger one, up to the dense windows (a row's result does not depend
// on the kernel that forms it); dense windows too wide for the budget give
// way to the narrowest (more passes per row); symbolic hash tables too large
// send their rows to the bitmap pass, whose bitmap also stays within it.
template <class SR> Schedule budgeted(const Ctx *c, int id) {
  Schedule S = schedule(id);
  const int64_t B = c->lds_budget;
  if (B >= LDS_BYTES) return S;
  if (sym_hash_lds<512>(16384) > B) S.sym_hash_max = std::min<int64_t>(S.sym_hash_max, 2048);
  if (sym_hash_lds<256>(4096) > B) S.sym_hash_max = std::min<int64_t>(S.sym_hash_max, 256);
  if (sym_hash_lds<64>(512) > B) S.sym_hash_max = std::min<int64_t>(S.sym_hash_max, 32);
  if (sym_hash_lds<64>(64) > B) S.sym_hash_max = 0;
  // numeric bins, largest first: a dropped bin's rows fall through to the
  // dense windows (thresholds are applied as running maxima)
  if (num_hash_lds<SR, 512>(8192) > B) S.t_big = S.t_mid;
  if (num_hash_lds<SR, 256>(4096) > B) S.t_mid = S.t_big = S.t_small;
  if (num_hash_lds<SR, 128>(512) > B) S.t_small = S.t_mid = S.t_big = S.t_tiny;
  if (num_hash_lds<SR, 64>(64) > B) S.t_tiny = S.t_small = S.t_mid = S.t_big = 0;
  constexpr int W0 = (int)dense_width<SR>(0), W1 = (int)dense_width<SR>(1), W2 = (int)dense_width<SR>(2);
  int need = 0;
  if (S.dense_wide == 1) need = num_dense_lds<SR, 1024, W1>();
  else if (S.dense_wide == 2) need = num_dense_lds<SR, 512, W2>();
  else need = S.dense_bs == 512 ? num_dense_lds<SR, 512, W0>() : num_dense_lds<SR, 256, W0>();
  if (need > B) {
    S.dense_wide = 2;
    S.dense_bs = 512;
    if (num_dense_lds<SR, 512, W2>() > B)
      fail(SRTC_ERR_UNSUPPORTED, "SRTC_LDS_BUDGET is below the narrowest dense window (" +
                                     std::to_string(num_dense_lds<SR, 512, W2>()) + " bytes)");
  }
  return S;
}

// Numeric binning of one group of rows (row ids in g.row_map, or every row
// when it is null) under schedule g.sched: rows go to bins by their exact
// output counts (info2: INFO entries, zeroed by the caller; list: the
// group's rows by bin).  Nothing is read back here.
template <class SR>
void numeric_bin(Ctx *c, const CsrView &Am, const int64_t *nnz_row, const RowGroup &g, int64_t *info2, int32_t *list,
                 Buf *vbuf, hipStream_t s) {
  const Schedule S = budgeted<SR>(c, g.sched);
  const int64_t nsel = g.row_map ? g.nsel : Am.m;
  if (nsel == 0) return;
  // output counts in selection order
  const int64_t *vsel = nnz_row;
  if (g.row_map) {
    *vbuf = Buf(c, sizeof(int64_t) * (size_t)nsel);
    gather_i64<<<gridn(nsel), 256, 0, s>>>(nnz_row, g.row_map, nsel, vbuf->as<int64_t>());
    SRTC_LAUNCH_CHECK("gather_i64");
    vsel = vbuf->as<int64_t>();
  }
  Thresholds th2{};
  th2.t[0] = S.t_tiny;
  th2.t[1] = std::max(S.t_small, th2.t[0]);
  th2.t[2] = std::max(S.t_mid, th2.t[1]);
  th2.t[3] = std::max(S.t_big, th2.t[2]);
  bin_count<<<gridn(nsel, 256, 2048), 256, 0, s>>>(vsel, nsel, th2, info2, Am.rowptr, g.row_map);
  SRTC_LAUNCH_CHECK("bin_count");
  bin_offsets<<<1, 64, 0, s>>>(info2);
  bin_scatter<<<gridn(nsel, 256, 4096), 256, 0, s>>>(vsel, nsel, th2, info2, list, g.row_map);
  SRTC_LAUNCH_CHECK("bin_scatter");
}

// Numeric kernels of one binned group (hinfo2: the host copy of its bin
// table), writing at rpC.  kp[row] = entries written; fl[0] is raised when a
// row came out short (identity results dropped) or holds an entry with
// column -1 (an identity result written in place), fl[1] on a broken hash
// invariant.
template <class SR>
void numeric_launch(Ctx *c, typename SR::acc_t id, const CsrView &Am, const CsrView &Bm, const int64_t *w,
                    const RowGroup &g, const int64_t *hinfo2, int64_t *info2, int32_t *lst, int sorted,
                    OutRows rpC, int32_t *cC, typename SR::val_t *vC, int64_t *kp, int32_t *fl,
                    SpgemmStats *st, hipStream_t s) {
  using V = typename SR::val_t;
  const Schedule S = budgeted<SR>(c, g.sched);
  const int64_t n = Bm.n;
  Launch L{c, s};
  heavy_first(c, lst + hinfo2[NBIN + 5], hinfo2[5], w, s);
  c->tracef("spgemm: schedule %d, nnz %lld; numeric bins %lld %lld %lld %lld %lld", g.sched,
            (long long)hinfo2[4 * NBIN], (long long)hinfo2[1], (long long)hinfo2[2], (long long)hinfo2[3],
            (long long)hinfo2[4], (long long)hinfo2[5]);
  if (st) st->dense_rows += hinfo2[5];
  int64_t *ctr2 = info2 + 3 * NBIN;
  using NL = NumLaunch<SR>;
  // algorithmic bytes of a numeric bin: its C entries written, its A rows
  // read, B read once
  const double vb = (double)sizeof(V);
  auto num_bytes = [&](int b) {
    return (4.0 + vb) * hinfo2[SUMV + b] + (4.0 + vb) * hinfo2[SUMA + b] + 24.0 * hinfo2[b] +
           (4.0 + vb) * Bm.nnz + 8.0 * (Bm.m + 1);
  };
  static const char *kNumName[NBIN] = {"", "spgemm.numeric.hash64", "spgemm.numeric.hash512",
                                       "spgemm.numeric.hash4096", "spgemm.numeric.hash8192",
                                       "spgemm.numeric.dense"};
  // profile names carry the value type, so each names one kernel instance
  const char *vt = std::is_same<V, double>::value ? ".f64" : std::is_same<V, float>::value ? ".f32"
                   : std::is_same<V, int32_t>::value ? ".i32" : std::is_same<V, uint64_t>::value ? ".path" : ".u8";
  auto pname = [&](int b) { return std::string(kNumName[b]) + vt; };
  for (int b = 1; b < NBIN - 1; b++) {
    if (hinfo2[b] == 0) continue;
    ProfScope ps(c, pname(b).c_str(), num_bytes(b), s);
    if (b == 1) {
      if (sorted) NL::template hash<64, 64, 0>(L, hinfo2[1], lst, info2, 1, Am, Bm, rpC, cC, vC, id, kp, fl, ctr2 + 1);
      else NL::template hash<64, 64, 2>(L, hinfo2[1], lst, info2, 1, Am, Bm, rpC, cC, vC, id, kp, fl, ctr2 + 1);
    } else if (b == 2) {
      if (!sorted) NL::template hash<128, 512, 2>(L, hinfo2[2], lst, info2, 2, Am, Bm, rpC, cC, vC, id, kp, fl, ctr2 + 2);
      else if (S.small_wave) NL::template hash<64, 512, 0>(L, hinfo2[2], lst, info2, 2, Am, Bm, rpC, cC, vC, id, kp, fl, ctr2 + 2);
      else NL::template hash<128, 512, 0>(L, hinfo2[2], lst, info2, 2, Am, Bm, rpC, cC, vC, id, kp, fl, ctr2 + 2);
    } else if (b == 3) {
      if (sorted) NL::template hash<256, 4096, 0>(L, hinfo2[3], lst, info2, 3, Am, Bm, rpC, cC, vC, id, kp, fl, ctr2 + 3);
      else NL::template hash<256, 4096, 2>(L, hinfo2[3], lst, info2, 3, Am, Bm, rpC, cC, vC, id, kp, fl, ctr2 + 3);
    } else {
      if (sorted) NL::template hash<512, 8192, 0>(L, hinfo2[4], lst, info2, 4, Am, Bm, rpC, cC, vC, id, kp, fl, ctr2 + 4);
      else NL::template hash<512, 8192, 2>(L, hinfo2[4], lst, info2, 4, Am, Bm, rpC, cC, vC, id, kp, fl, ctr2 + 4);
    }
  }
  if (hinfo2[5] > 0) {
    const int64_t W = dense_width<SR>(S.dense_wide);
    const int nwin = (int)((n + W - 1) / W);
    Buf woff;
    const int32_t *wo = nullptr;
    if (nwin > 1)
      wo = (const int32_t *)b_table(c, Bm, W, sizeof(int32_t) * (size_t)(Bm.m * (nwin + 1)), woff, [&](void *d) {
        ProfScope ps(c, "spgemm.window_table", 8.0 * (Bm.m + 1) + 4.0 * Bm.nnz + 4.0 * Bm.m * (nwin + 1), s);
        build_woff<<<gridn(Bm.m * (nwin + 1)), 256, 0, s>>>(Bm.rowptr, Bm.col, Bm.m, nwin, W, (int32_t *)d);
        SRTC_LAUNCH_CHECK("build_woff");
      });
    Buf recs;
    const uint2 *rb = nullptr;
    if constexpr (b_records<SR>())
      rb = (const uint2 *)b_table(c, Bm, -1, sizeof(uint2) * (size_t)std::max<int64_t>(Bm.nnz, 1), recs, [&](void *d) {
        ProfScope pr(c, "spgemm.b_records", 16.0 * Bm.nnz, s);
        pack_records<V><<<gridn(Bm.nnz), 256, 0, s>>>(Bm.rowptr, Bm.col, (const V *)Bm.val, Bm.nnz, (uint2 *)d);
        SRTC_LAUNCH_CHECK("pack_records");
      });
    // the window-table lookups (8 B per A entry and window) are overhead of
    // the method, not bytes the product must move: they stay out of the count
    ProfScope ps(c, pname(5).c_str(), num_bytes(5), s);
    constexpr int W0 = (int)dense_width<SR>(0), W1 = (int)dense_width<SR>(1), W2 = (int)dense_width<SR>(2);
    if (S.dense_wide == 1) {
      // the widest window fills the LDS (one block per CU): 1024 threads keep
      // 16 waves per CU in flight instead of 8
      NL::template dense<1024, W1>(L, hinfo2[5], lst, info2, 5, Am, Bm, wo, nwin, rb, rpC, cC, vC, id, kp, fl, ctr2 + 5);
    } else if (S.dense_wide == 2) {
      NL::template dense<512, W2>(L, hinfo2[5], lst, info2, 5, Am, Bm, wo, nwin, rb, rpC, cC, vC, id, kp, fl, ctr2 + 5);
    } else {
      if (S.dense_bs == 512) NL::template dense<512, W0>(L, hinfo2[5], lst, info2, 5, Am, Bm, wo, nwin, rb, rpC, cC, vC, id, kp, fl, ctr2 + 5);
      else NL::template dense<256, W0>(L, hinfo2[5], lst, info2, 5, Am, Bm, wo, nwin, rb, rpC, cC, vC, id, kp, fl, ctr2 + 5);
    }
  }
}

__global__ void copy_i64(const int64_t *src, int64_t *dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

// C = A (x) B with the rows split into groups, each multiplied under its own
// schedule (one group of every row for a plain product).  The symbolic
// counts do not depend on the schedule, so one row pointer array and one
// output allocation serve every group.  Host reads: each group's symbolic
// bin sizes, then the output size with every group's numeric bin sizes,
// then the end-of-product flags.
template <class SR>
void spgemm_groups(Ctx *c, IdVal idv, const CsrView &Am, const CsrView &Bm, const std::vector<RowGroup> &groups,
                   int sorted, CsrOut *out, SpgemmStats *st, hipStream_t s) {
  using V = typename SR::val_t;
  using A = typename SR::acc_t;
  const A id = id_as<SR>(idv);
  const int64_t m = Am.m;
  Launch L{c, s};
  out->m = m;
  out->n = Bm.n;
  out->rowptr = Buf(c, sizeof(int64_t) * (size_t)(m + 1), out->kind);
  const size_t es = sizeof(V);
  if (st) *st = SpgemmStats{};
  if (m == 0 || Am.nnz == 0 || Bm.nnz == 0) {
    fill_i64(out->rowptr.as<int64_t>(), m + 1, 0, s);
    out->nnz = 0;
    out->col = Buf(c, 4, out->kind);
    out->val = Buf(c, es, out->kind);
    return;
  }
  const int G = (int)groups.size();
  // flags: [0] a row came out short, [1] numeric hash invariant broken,
  // int64 at byte 8: symbolic hash invariant broken
  Buf flag(c, 64);
  fill_i32(flag.as<int32_t>(), 4, 0, s);
  int32_t *fl = flag.as<int32_t>();
  int64_t *sym_err = reinterpret_cast<int64_t *>(flag.as<char>() + 8);
  // 1-3. products per row, symbolic bins, symbolic pass (per group)
  Buf w(c, sizeof(int64_t) * (size_t)m);
  {
    ProfScope ps(c, "spgemm.row_products", 16.0 * (m + 1) + 4.0 * Am.nnz + 8.0 * (Bm.m + 1), s);
    row_products(Am, Bm, w.as<int64_t>(), s);
  }
  Buf nnz_row(c, sizeof(int64_t) * (size_t)m);
  fill_i64(nnz_row.as<int64_t>(), m, 0, s);
  c->tracef("spgemm: %lld x %lld (nnz %lld) times %lld x %lld (nnz %lld), %d group(s), schedule %d", (long long)m,
            (long long)Am.n, (long long)Am.nnz, (long long)Bm.m, (long long)Bm.n, (long long)Bm.nnz, G,
            G ? groups[0].sched : -1);
  // per group: a bin table (symbolic, then reused for the numeric pass) and
  // a row list; slot 0 of `tables` receives the output size
  Buf tables(c, sizeof(int64_t) * (size_t)(1 + G * INFO));
  int64_t *tab = tables.as<int64_t>();
  fill_i64(tab, 1 + (int64_t)G * INFO, 0, s);
  std::vector<Buf> lists(G);
  int64_t products = 0;
  for (int q = 0; q < G; q++) {
    const RowGroup &g = groups[q];
    const int64_t nsel = g.row_map ? g.nsel : m;
    lists[q] = Buf(c, sizeof(int32_t) * (size_t)std::max<int64_t>(nsel, 1));
    if (nsel == 0) continue;
    int64_t *info1 = tab + 1 + (int64_t)q * INFO;
    products += run_symbolic(L, budgeted<SR>(c, g.sched), Am, Bm, w.as<int64_t>(), g.row_map, nsel, info1,
                             lists[q].as<int32_t>(), nnz_row.as<int64_t>(), sym_err);
    fill_i64(info1, INFO, 0, s);  // the table serves the numeric binning next
  }
  c->tracef("spgemm: symbolic launched, %lld products", (long long)products);
  if (st) st->products = products;
  // 4. rowptr of C, numeric bins; one host read sizes C and every bin
  excl_scan_i64(c, nnz_row.as<int64_t>(), out->rowptr.as<int64_t>(), m, s);
  std::vector<Buf> vbufs(G);
  for (int q = 0; q < G; q++)
    numeric_bin<SR>(c, Am, nnz_row.as<int64_t>(), groups[q], tab + 1 + (int64_t)q * INFO, lists[q].as<int32_t>(),
                    &vbufs[q], s);
  copy_i64<<<1, 64, 0, s>>>(out->rowptr.as<int64_t>() + m, tab);
  std::vector<int64_t> htab(1 + (size_t)G * INFO);
  read_to_host(c, htab.data(), tab, sizeof(int64_t) * htab.size(), s);
  const int64_t total = htab[0];
  c->tracef("spgemm: nnz(C) = %lld", (long long)total);
  if (st) st->nnz = total;
  // 5. numeric, group by group into the one output
  Buf col(c, sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1), out->kind);
  Buf val(c, es * (size_t)std::max<int64_t>(total, 1), out->kind);
  Buf kept(c, sizeof(int64_t) * (size_t)m);
  fill_i64(kept.as<int64_t>(), m, 0, s);  // rows in no bin (no outputs) keep 0
  const int64_t *rpC = out->rowptr.as<int64_t>();
  int32_t *cC = col.as<int32_t>();
  V *vC = val.as<V>();
  int64_t *kp = kept.as<int64_t>();
  if (total > 0)
    for (int q = 0; q < G; q++)
      numeric_launch<SR>(c, id, Am, Bm, w.as<int64_t>(), groups[q], htab.data() + 1 + (size_t)q * INFO,
                         tab + 1 + (int64_t)q * INFO, lists[q].as<int32_t>(), sorted,
                         OutRows{rpC, nnz_row.as<int64_t>(), 0}, cC, vC, kp, fl, st, s);
  // 6. compaction when identity results were dropped
  int32_t flags_h[4] = {0, 0, 0, 0};
  read_to_host(c, flags_h, fl, sizeof(flags_h), s);
  c->tracef("spgemm: numeric done (short %d, error %d)", flags_h[0], flags_h[1]);
  if (flags_h[2] || flags_h[3]) fail(SRTC_ERR_DEVICE, "spgemm: symbolic hash table overflow (internal invariant)");
  if (flags_h[1]) fail(SRTC_ERR_DEVICE, "spgemm: numeric hash table overflow (internal invariant)");
  const int32_t short_flag = flags_h[0];
  if (short_flag) {
    // identity results were dropped or marked: count each row's kept
    // entries among the kp[i] written, then pack them
    Buf kv(c, sizeof(int64_t) * (size_t)m);
    count_valid<<<gridn(m * WAVE, 256, 16384), 256, 0, s>>>(nullptr, m, 1, m, rpC, kp, cC, kv.as<int64_t>());
    SRTC_LAUNCH_CHECK("count_valid");
    Buf rp2(c, sizeof(int64_t) * (size_t)(m + 1), out->kind);
    excl_scan_i64(c, kv.as<int64_t>(), rp2.as<int64_t>(), m, s);
    const int64_t t2 = read_i64(c, rp2.as<int64_t>() + m, s);
    Buf col2(c, sizeof(int32_t) * (size_t)std::max<int64_t>(t2, 1), out->kind);
    Buf val2(c, es * (size_t)std::max<int64_t>(t2, 1), out->kind);
    compact_valid<V><<<gridn(m * WAVE, 256, 16384), 256, 0, s>>>(nullptr, m, 1, m, rpC, kp, rp2.as<int64_t>(), cC,
                                                                  vC, col2.as<int32_t>(), val2.as<V>());
    SRTC_LAUNCH_CHECK("compact_valid");
    out->rowptr = std::move(rp2);
    col = std::move(col2);
    val = std::move(val2);
    if (st) { st->nnz = t2; st->compacted = 1; }
    out->nnz = t2;
  } else {
    out->nnz = total;
  }
  out->col = std::move(col);
  out->val = std::move(val);
}

// ------------------------------------------------ column blocks of B --
// For products whose B is far larger than the caches, the rows with many
// products are multiplied one column block of B at a time: block q holds B's
// entries with columns in [q bc, (q+1) bc) as a CSR over B's rows with
// block-local columns.  A heavy row's products in block q then gather from a
// slice of B that stays cache-resident while every heavy row passes through
// that block, instead of re-reading B's lines from HBM once per dense window
// (B's rows are short and spread over every window).  C's row i is the
// concatenation of its blocks' results, so block q of row i is written at
// rowptr[i] + (outputs of row i in blocks before q).

// cnt[q (K+1) + k] = entries of row k of B in block q (the slot k = K stays 0).
__global__ void colblock_count(const int64_t *__restrict__ rpB, const int32_t *__restrict__ cB, int64_t K, int Q,
                               int64_t bc, int64_t *__restrict__ cnt) {
  const int64_t total = K * Q;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / Q;
    const int q = (int)(t % Q);
    const int64_t a = rpB[k], b = rpB[k + 1];
    auto lower = [&](int64_t target) {
      int64_t lo = a, hi = b;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cB[mid] < target) lo = mid + 1; else hi = mid;
      }
      return lo;
    };
    cnt[(int64_t)q * (K + 1) + k] = lower((int64_t)(q + 1) * bc) - lower((int64_t)q * bc);
  }
}

// Entry e of row k goes to block q = col / bc at pos[q (K+1) + k] + its rank
// among the row's entries of that block (the row is column-sorted, so the
// block's entries are consecutive: rank = e - first entry with col >= q bc).
template <class V>
__global__ void colblock_scatter(const int64_t *__restrict__ rpB, const int32_t *__restrict__ cB,
                                 const V *__restrict__ vB, int64_t K, int64_t bc, int Q,
                                 const int64_t *__restrict__ pos, int32_t *__restrict__ col, V *__restrict__ val,
                                 bool vals) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t k = wid; k < K; k += nw) {
    const int64_t a = rpB[k], b = rpB[k + 1];
    for (int64_t e = a + lane_id(); e < b; e += WAVE) {
      const int32_t c = cB[e];
      const int64_t q = c / bc;
      if (c < 0 || q >= Q) continue;  // outside the columns (a malformed operand): counted by no block
      const int64_t target = q * bc;
      int64_t lo = a, hi = e;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cB[mid] < target) lo = mid + 1; else hi = mid;
      }
      const int64_t d = pos[q * (K + 1) + k] + (e - lo);
      col[d] = (int32_t)(c - target);
      if (vals) val[d] = vB[e];
    }
  }
}

// Rows with at least thr products go to `heavy`, the others to `light`
// (ballot ranks, one atomic per wave and list); counts in ctr[0], ctr[1].
__global__ void split_rows(const int64_t *__restrict__ w, int64_t m, int64_t thr, int32_t *__restrict__ light,
                           int32_t *__restrict__ heavy, unsigned long long *__restrict__ ctr) {
  const uint64_t lt = lanemask_lt();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < m; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    const bool in = i < m;
    const bool h = in && w[i] >= thr;
#pragma unroll
    for (int s = 0; s < 2; s++) {
      const bool mine = in && (s == 1 ? h : !h);
      const uint64_t mk = __ballot(mine);
      if (mk == 0) continue;
      const int leader = __ffsll((unsigned long long)mk) - 1;
      unsigned long long p = 0;
      if (lane_id() == leader) p = atomicAdd(&ctr[s], (unsigned long long)__popcll(mk));
      p = __shfl(p, leader, WAVE);
      if (mine) (s == 1 ? heavy : light)[p + __popcll(mk & lt)] = (int32_t)i;
    }
  }
}

// Products per listed row (row_products restricted to a row list).
__global__ void row_products_rows(const int64_t *__restrict__ rpA, const int32_t *__restrict__ cA,
                                  const int64_t *__restrict__ rpB, const int32_t *__restrict__ rows, int64_t n,
                                  int64_t *__restrict__ w) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t r = wid; r < n; r += nw) {
    const int64_t i = rows[r];
    int64_t acc = 0;
    for (int64_t p = rpA[i] + lane_id(); p < rpA[i + 1]; p += WAVE) {
      const int32_t k = cA[p];
      acc += rpB[k + 1] - rpB[k];
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) w[i] = acc;
  }
}

// Per heavy row: total over blocks (tot[i]), and with rowptr given, every
// block's first output position (start[q m + i]).
__global__ void block_rows(const int32_t *__restrict__ rows, int64_t n, const int64_t *__restrict__ cnt, int Q,
                           int64_t m, int64_t *__restrict__ tot, const int64_t *__restrict__ rp,
                           int64_t *__restrict__ start) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = rows[r];
    int64_t run = rp ? rp[i] : 0;
    for (int q = 0; q < Q; q++) {
      if (start) start[(int64_t)q * m + i] = run;
      run += cnt[(int64_t)q * m + i];
    }
    if (tot) tot[i] = rp ? run - rp[i] : run;
  }
}


// C = A (x) B with B cut into Q column blocks of bc columns for the rows of
// at least thr products (the others multiply the whole B once).  Host reads:
// the row split and block sizes, each symbolic pass's bins, the output size
// with every numeric bin table, the flags.
template <class SR>
void spgemm_blocked(Ctx *c, IdVal idv, const CsrView &Am, const CsrView &Bm, int sched, int Q, int64_t bc,
                    int64_t thr, const int64_t *w, int sorted, CsrOut *out, SpgemmStats *st, hipStream_t s) {
  using V = typename SR::val_t;
  using A = typename SR::acc_t;
  const A id = id_as<SR>(idv);
  const int64_t m = Am.m, K = Bm.m;
  const size_t es = sizeof(V);
  Launch L{c, s};
  c->tracef("spgemm: %lld x %lld (nnz %lld) times %lld x %lld (nnz %lld), schedule %d, %d column blocks of %lld",
            (long long)m, (long long)Am.n, (long long)Am.nnz, (long long)K, (long long)Bm.n, (long long)Bm.nnz, sched,
            Q, (long long)bc);
  // B's column blocks, one shared entry array
  Buf pos(c, sizeof(int64_t) * (size_t)(Q * (K + 1) + 1));
  Buf bcol(c, sizeof(int32_t) * (size_t)std::max<int64_t>(Bm.nnz, 1));
  Buf bval(c, es * (size_t)(SR::HAS_VALS ? std::max<int64_t>(Bm.nnz, 1) : 1));
  {
    ProfScope ps(c, "spgemm.column_blocks", 16.0 * (K + 1) + (8.0 + 2.0 * es) * Bm.nnz + 8.0 * Q * (K + 1), s);
    Buf cnt(c, sizeof(int64_t) * (size_t)(Q * (K + 1)));
    fill_i64(cnt.as<int64_t>(), Q * (K + 1), 0, s);
    colblock_count<<<gridn(K * Q), 256, 0, s>>>(Bm.rowptr, Bm.col, K, Q, bc, cnt.as<int64_t>());
    SRTC_LAUNCH_CHECK("colblock_count");
    excl_scan_i64(c, cnt.as<int64_t>(), pos.as<int64_t>(), Q * (K + 1), s);
    colblock_scatter<V><<<gridn(K * WAVE, 256, 16384), 256, 0, s>>>(Bm.rowptr, Bm.col, (const V *)Bm.val, K, bc, Q,
                                                                     pos.as<int64_t>(), bcol.as<int32_t>(),
                                                                     bval.as<V>(), SR::HAS_VALS);
    SRTC_LAUNCH_CHECK("colblock_scatter");
  }
  // rows: light (whole B) and heavy (block by block)
  Buf lists(c, sizeof(int32_t) * (size_t)(2 * m));
  int32_t *light = lists.as<int32_t>(), *heavy = light + m;
  Buf ctr(c, 64);
  fill_i64(ctr.as<int64_t>(), 2, 0, s);
  split_rows<<<gridn(m, 256, 4096), 256, 0, s>>>(w, m, thr, light, heavy, (unsigned long long *)ctr.p);
  SRTC_LAUNCH_CHECK("split_rows");
  std::vector<int64_t> hb(2 + Q + 1);
  {
    // the split sizes and each block's first entry, in one read
    Buf bounds(c, sizeof(int64_t) * (size_t)(Q + 3));
    SRTC_HIP(hipMemcpyAsync(bounds.p, ctr.p, 16, hipMemcpyDeviceToDevice, s));
    for (int q = 0; q <= Q; q++)
      copy_i64<<<1, 64, 0, s>>>(pos.as<int64_t>() + (int64_t)q * (K + 1), bounds.as<int64_t>() + 2 + q);
    read_to_host(c, hb.data(), bounds.p, sizeof(int64_t) * hb.size(), s);
  }
  const int64_t nlight = hb[0], nheavy = hb[1];
  auto block_view = [&](int q) {
    const int64_t b0 = (int64_t)q * bc;
    return CsrView{K, std::min(bc, Bm.n - b0), hb[2 + q + 1] - hb[2 + q], pos.as<int64_t>() + (int64_t)q * (K + 1),
                   bcol.as<int32_t>(), bval.p};
  };
  // groups: [0] light rows against B, [1 + q] heavy rows against block q
  const int G = 1 + Q;
  std::vector<RowGroup> grp(G);
  grp[0] = RowGroup{light, nlight, sched};
  for (int q = 0; q < Q; q++) grp[1 + q] = RowGroup{heavy, nheavy, sched};
  // products per heavy row and block, output counts per row and block
  Buf wq(c, sizeof(int64_t) * (size_t)(Q * m));
  Buf nnzq(c, sizeof(int64_t) * (size_t)(Q * m));
  Buf nnz_row(c, sizeof(int64_t) * (size_t)m);
  fill_i64(nnz_row.as<int64_t>(), m, 0, s);
  fill_i64(nnzq.as<int64_t>(), Q * m, 0, s);
  Buf flag(c, 64);
  fill_i32(flag.as<int32_t>(), 4, 0, s);
  int32_t *fl = flag.as<int32_t>();
  int64_t *sym_err = reinterpret_cast<int64_t *>(flag.as<char>() + 8);
  Buf tables(c, sizeof(int64_t) * (size_t)(1 + G * INFO));
  int64_t *tab = tables.as<int64_t>();
  fill_i64(tab, 1 + (int64_t)G * INFO, 0, s);
  std::vector<Buf> blists(G);
  int64_t products = 0;
  for (int q = 0; q < G; q++) {
    const RowGroup &g = grp[q];
    blists[q] = Buf(c, sizeof(int32_t) * (size_t)std::max<int64_t>(g.nsel, 1));
    if (g.nsel == 0) continue;
    int64_t *info1 = tab + 1 + (int64_t)q * INFO;
    if (q == 0) {
      products += run_symbolic(L, budgeted<SR>(c, sched), Am, Bm, w, light, nlight, info1, blists[q].as<int32_t>(),
                               nnz_row.as<int64_t>(), sym_err);
    } else {
      const CsrView bq = block_view(q - 1);
      int64_t *wq_b = wq.as<int64_t>() + (int64_t)(q - 1) * m;
      row_products_rows<<<gridn(nheavy * WAVE, 256, 16384), 256, 0, s>>>(Am.rowptr, Am.col, bq.rowptr, heavy, nheavy,
                                                                         wq_b);
      SRTC_LAUNCH_CHECK("row_products_rows");
      products += run_symbolic(L, budgeted<SR>(c, sched), Am, bq, wq_b, heavy, nheavy, info1,
                               blists[q].as<int32_t>(), nnzq.as<int64_t>() + (int64_t)(q - 1) * m, sym_err);
    }
    fill_i64(info1, INFO, 0, s);
  }
  if (st) st->products = products;
  // rowptr: heavy rows' totals over blocks, then the scan; block starts
  Buf startq(c, sizeof(int64_t) * (size_t)(Q * m));
  if (nheavy > 0) {
    block_rows<<<gridn(nheavy), 256, 0, s>>>(heavy, nheavy, nnzq.as<int64_t>(), Q, m, nnz_row.as<int64_t>(), nullptr,
                                            nullptr);
    SRTC_LAUNCH_CHECK("block_rows");
  }
  excl_scan_i64(c, nnz_row.as<int64_t>(), out->rowptr.as<int64_t>(), m, s);
  const int64_t *rpC = out->rowptr.as<int64_t>();
  if (nheavy > 0) {
    block_rows<<<gridn(nheavy), 256, 0, s>>>(heavy, nheavy, nnzq.as<int64_t>(), Q, m, nullptr, rpC,
                                            startq.as<int64_t>());
    SRTC_LAUNCH_CHECK("block_rows");
  }
  std::vector<Buf> vbufs(G);
  for (int q = 0; q < G; q++)
    numeric_bin<SR>(c, Am, q == 0 ? nnz_row.as<int64_t>() : nnzq.as<int64_t>() + (int64_t)(q - 1) * m, grp[q],
                    tab + 1 + (int64_t)q * INFO, blists[q].as<int32_t>(), &vbufs[q], s);
  copy_i64<<<1, 64, 0, s>>>(rpC + m, tab);
  std::vector<int64_t> htab(1 + (size_t)G * INFO);
  read_to_host(c, htab.data(), tab, sizeof(int64_t) * htab.size(), s);
  const int64_t total = htab[0];
  c->tracef("spgemm: %lld light and %lld heavy rows, %lld products, nnz(C) = %lld", (long long)nlight,
            (long long)nheavy, (long long)products, (long long)total);
  if (st) st->nnz = total;
  Buf col(c, sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1), out->kind);
  Buf val(c, es * (size_t)std::max<int64_t>(total, 1), out->kind);
  Buf kept(c, sizeof(int64_t) * (size_t)m), keptq(c, sizeof(int64_t) * (size_t)(Q * m));
  fill_i64(kept.as<int64_t>(), m, 0, s);
  fill_i64(keptq.as<int64_t>(), Q * m, 0, s);
  int32_t *cC = col.as<int32_t>();
  V *vC = val.as<V>();
  if (total > 0) {
    for (int q = 0; q < G; q++) {
      if (grp[q].nsel == 0) continue;
      if (q == 0) {
        numeric_launch<SR>(c, id, Am, Bm, w, grp[0], htab.data() + 1, tab + 1, blists[0].as<int32_t>(), sorted,
                           OutRows{rpC, nnz_row.as<int64_t>(), 0}, cC, vC, kept.as<int64_t>(), fl, st, s);
      } else {
        const int64_t off = (int64_t)(q - 1) * m;
        numeric_launch<SR>(c, id, Am, block_view(q - 1), wq.as<int64_t>() + off, grp[q],
                           htab.data() + 1 + (size_t)q * INFO, tab + 1 + (int64_t)q * INFO, blists[q].as<int32_t>(),
                           sorted, OutRows{startq.as<int64_t>() + off, nnzq.as<int64_t>() + off, (q - 1) * bc}, cC, vC,
                           keptq.as<int64_t>() + off, fl, st, s);
      }
    }
  }
  int32_t flags_h[4] = {0, 0, 0, 0};
  read_to_host(c, flags_h, fl, sizeof(flags_h), s);
  c->tracef("spgemm: numeric done (short %d, error %d)", flags_h[0], flags_h[1]);
  if (flags_h[2] || flags_h[3]) fail(SRTC_ERR_DEVICE, "spgemm: symbolic hash table overflow (internal invariant)");
  if (flags_h[1]) fail(SRTC_ERR_DEVICE, "spgemm: numeric hash table overflow (internal invariant)");
  if (flags_h[0]) {
    // identity results were dropped or marked: each row's kept entries
    // over its segments (one for light rows, one per block for heavy ones),
    // then every segment's kept entries move to their packed place
    Buf kv(c, sizeof(int64_t) * (size_t)m);
    fill_i64(kv.as<int64_t>(), m, 0, s);
    if (nlight > 0)
      count_valid<<<gridn(nlight * WAVE, 256, 16384), 256, 0, s>>>(light, nlight, 1, m, rpC, kept.as<int64_t>(), cC,
                                                                  kv.as<int64_t>());
    if (nheavy > 0)
      count_valid<<<gridn(nheavy * WAVE, 256, 16384), 256, 0, s>>>(heavy, nheavy, Q, m, startq.as<int64_t>(),
                                                                  keptq.as<int64_t>(), cC, kv.as<int64_t>());
    SRTC_LAUNCH_CHECK("count_valid");
    Buf rp2(c, sizeof(int64_t) * (size_t)(m + 1), out->kind);
    excl_scan_i64(c, kv.as<int64_t>(), rp2.as<int64_t>(), m, s);
    const int64_t t2 = read_i64(c, rp2.as<int64_t>() + m, s);
    Buf col2(c, sizeof(int32_t) * (size_t)std::max<int64_t>(t2, 1), out->kind);
    Buf val2(c, es * (size_t)std::max<int64_t>(t2, 1), out->kind);
    if (nlight > 0)
      compact_valid<V><<<gridn(nlight * WAVE, 256, 16384), 256, 0, s>>>(light, nlight, 1, m, rpC, kept.as<int64_t>(),
                                                                         rp2.as<int64_t>(), cC, vC,
                                                                         col2.as<int32_t>(), val2.as<V>());
    if (nheavy > 0)
      compact_valid<V><<<gridn(nheavy * WAVE, 256, 16384), 256, 0, s>>>(heavy, nheavy, Q, m, startq.as<int64_t>(),
                                                                         keptq.as<int64_t>(), rp2.as<int64_t>(), cC,
                                                                         vC, col2.as<int32_t>(), val2.as<V>());
    SRTC_LAUNCH_CHECK("compact_valid");
    out->rowptr = std::move(rp2);
    col = std::move(col2);
    val = std::move(val2);
    if (st) { st->nnz = t2; st->compacted = 1; }
    out->nnz = t2;
  } else {
    out->nnz = total;
  }
  out->col = std::move(col);
  out->val = std::move(val);
}

// Column blocking (above) is opt-in (SRTC_COL_BLOCKS): on the R-MAT 21
// square it moved B's gathers off HBM, but the dense-window kernel is bound
// by its per-window work, not by those bytes (8% faster), while rows split
// over blocks fell into slower hash bins and the block copies cost more
// than that.  Blocks then hold about kBlockBytes of B each.
constexpr int64_t kBlockBytes = 48ll << 20;

template <class SR>
void spgemm_typed(Ctx *c, IdVal idv, const CsrView &Am, const CsrView &Bm, const std::vector<RowGroup> *groups,
                  int sched, int sorted, CsrOut *out, SpgemmStats *st, hipStream_t s) {
  if (groups) {
    spgemm_groups<SR>(c, idv, Am, Bm, *groups, sorted, out, st, s);
    return;
  }
  using V = typename SR::val_t;
  const Schedule S = budgeted<SR>(c, sched);
  const int64_t W = dense_width<SR>(S.dense_wide);
  const double eb = 4.0 + (SR::HAS_VALS ? (double)sizeof(V) : 0.0);
  // SRTC_COL_BLOCKS=0: blocks of whole dense windows, each about
  // kBlockBytes of B; SRTC_COL_BLOCKS=q >= 2: q blocks, a multiple of 32
  // columns each; unset: no blocks
  int Q = 1;
  int64_t align = W;
  if (c->col_blocks == 0) {
    Q = (int)std::min<double>(std::ceil(eb * (double)Bm.nnz / (double)kBlockBytes), (double)(Bm.n / W));
  } else if (c->col_blocks >= 2) {
    Q = std::min<int>(c->col_blocks, (int)std::max<int64_t>(1, Bm.n / 32));
    align = 32;
  }
  if (Q >= 2 && Am.m > 0 && Am.nnz > 0 && Bm.nnz > 0 && Bm.m < 0x7fffffff) {
    const int64_t bc = ((Bm.n + Q - 1) / Q + align - 1) / align * align;
    Q = (int)((Bm.n + bc - 1) / bc);
    const int64_t thr = (int64_t)Q * 2048;
    out->m = Am.m;
    out->n = Bm.n;
    out->rowptr = Buf(c, sizeof(int64_t) * (size_t)(Am.m + 1), out->kind);
    Buf w(c, sizeof(int64_t) * (size_t)Am.m);
    {
      ProfScope ps(c, "spgemm.row_products", 16.0 * (Am.m + 1) + 4.0 * Am.nnz + 8.0 * (Bm.m + 1), s);
      row_products(Am, Bm, w.as<int64_t>(), s);
    }
    spgemm_blocked<SR>(c, idv, Am, Bm, sched, Q, bc, thr, w.as<int64_t>(), sorted, out, st, s);
    return;
  }
  const std::vector<RowGroup> one{RowGroup{nullptr, Am.m, sched}};
  spgemm_groups<SR>(c, idv, Am, Bm, one, sorted, out, st, s);
}

// Row statistics for the schedule features: log2 histograms of row lengths
// of A and of row product counts, maxima, sums, empty rows.
__global__ void feat_stats_kernel(const int64_t *__restrict__ rpA, const int64_t *__restrict__ w, int64_t m,
                                  unsigned long long *__restrict__ hist, unsigned long long *__restrict__ mx,
                                  double *__restrict__ sums) {
  __shared__ unsigned long long h[21];
  __shared__ unsigned long long lmx[2];
  __shared__ double ls[2];
  if (threadIdx.x < 21) h[threadIdx.x] = 0;
  if (threadIdx.x < 2) { lmx[threadIdx.x] = 0; ls[threadIdx.x] = 0.0; }
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t nz = rpA[i + 1] - rpA[i];
    const int64_t wi = w[i];
    const int bn = nz == 0 ? 0 : min(9, 64 - __clzll((unsigned long long)nz));          // ceil-ish log2(nz+1)
    const int bw = wi == 0 ? 0 : min(9, (64 - __clzll((unsigned long long)wi) + 1) / 2);  // base-4 bins
    atomicAdd(&h[bn], 1ull);
    atomicAdd(&h[10 + bw], 1ull);
    if (wi == 0) atomicAdd(&h[20], 1ull);
    atomicMax(&lmx[0], (unsigned long long)wi);
    atomicMax(&lmx[1], (unsigned long long)nz);
    atomicAdd(&ls[0], (double)wi);
    atomicAdd(&ls[1], (double)wi * (double)wi);
  }
  __syncthreads();
  if (threadIdx.x < 21) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x < 2) {
    atomicMax(&mx[threadIdx.x], lmx[threadIdx.x]);
    atomicAdd(&sums[threadIdx.x], ls[threadIdx.x]);
  }
}

}  // namespace

const Schedule &schedule(int id) {
  if (id < 0 || id >= SRTC_NUM_SCHEDULES) fail(SRTC_ERR_ARG, "schedule id out of range");
  return kSchedules[id];
}

void row_products(const CsrView &A, const CsrView &B, int64_t *w, hipStream_t s) {
  if (A.m == 0) return;
  row_products_kernel<<<gridn(A.m * WAVE, 256, 16384), 256, 0, s>>>(A.rowptr, A.col, B.rowptr, A.m, w);
  SRTC_LAUNCH_CHECK("row_products");
}

template <class SR>
void masked_typed(Ctx *c, IdVal idv, const CsrView &Am, const CsrView &Bm, const CsrView &Mm, CsrOut *out,
                  hipStream_t s) {
  using V = typename SR::val_t;
  using A = typename SR::acc_t;
  const A id = id_as<SR>(idv);
  const int64_t m = Am.m;
  const size_t es = sizeof(V);
  out->m = m;
  out->n = Bm.n;
  if (m == 0 || Am.nnz == 0 || Bm.nnz == 0 || Mm.nnz == 0) {
    out->rowptr = Buf(c, sizeof(int64_t) * (size_t)(m + 1), out->kind);
    fill_i64(out->rowptr.as<int64_t>(), m + 1, 0, s);
    out->nnz = 0;
    out->col = Buf(c, 4, out->kind);
    out->val = Buf(c, es, out->kind);
    return;
  }
  constexpr int BS = 256, LM = 1024;  // short chunks: more items to balance, more blocks per CU
  Launch L{c, s};
  // work items: (row, chunk of LM mask entries)
  Buf cnt(c, sizeof(int64_t) * (size_t)m), ioff(c, sizeof(int64_t) * (size_t)(m + 1));
  masked_count_items<<<gridn(m), 256, 0, s>>>(Am.rowptr, Mm.rowptr, m, LM, cnt.as<int64_t>());
  SRTC_LAUNCH_CHECK("masked_count_items");
  excl_scan_i64(c, cnt.as<int64_t>(), ioff.as<int64_t>(), m, s);
  const int64_t items = read_i64(c, ioff.as<int64_t>() + m, s);
  out->rowptr = Buf(c, sizeof(int64_t) * (size_t)(m + 1), out->kind);
  if (items == 0) {
    fill_i64(out->rowptr.as<int64_t>(), m + 1, 0, s);
    out->nnz = 0;
    out->col = Buf(c, 4, out->kind);
    out->val = Buf(c, es, out->kind);
    return;
  }
  if (items >= 0x7fffffff) fail(SRTC_ERR_UNSUPPORTED, "masked spgemm: more than 2^31-2 work items");
  Buf irow(c, 4 * (size_t)items), ichunk(c, 4 * (size_t)items), order(c, 4 * (size_t)items);
  Buf witem(c, 8 * (size_t)items), src(c, 8 * (size_t)items), kept(c, 8 * (size_t)items);
  Buf koff(c, 8 * (size_t)(items + 1)), ctr(c, 64);
  {
    Buf w(c, sizeof(int64_t) * (size_t)m);
    row_products(Am, Bm, w.as<int64_t>(), s);
    masked_fill_items<<<gridn(m), 256, 0, s>>>(ioff.as<int64_t>(), Mm.rowptr, w.as<int64_t>(), m, LM,
                                                irow.as<int32_t>(), ichunk.as<int32_t>(), order.as<int32_t>(),
                                                witem.as<int64_t>(), src.as<int64_t>());
    SRTC_LAUNCH_CHECK("masked_fill_items");
    heavy_first(c, order.as<int32_t>(), items, witem.as<int64_t>(), s);
  }
  fill_i64(ctr.as<int64_t>(), 1, 0, s);
  Buf colM(c, sizeof(int32_t) * (size_t)Mm.nnz), valM(c, es * (size_t)Mm.nnz);
  {
    ProfScope ps(c, "spgemm.masked", 16.0 * (m + 1) + 12.0 * Am.nnz + (4.0 + es) * Bm.nnz + 4.0 * Mm.nnz +
                 (4.0 + es) * Mm.nnz, s);
    const int stat = LM * (4 + (int)sizeof(A)) + (int)sizeof(Chunk<BS, V>) + 64;
    masked_rows<SR, BS, LM><<<L.grid(items, stat, BS), BS, 0, s>>>(
        Am.rowptr, Am.col, (const V *)Am.val, Bm.rowptr, Bm.col, (const V *)Bm.val, Mm.rowptr, Mm.col,
        irow.as<int32_t>(), ichunk.as<int32_t>(), order.as<int32_t>(), items, colM.as<int32_t>(), valM.as<V>(), id,
        kept.as<int64_t>(), ctr.as<int64_t>());
    SRTC_LAUNCH_CHECK("masked_rows");
  }
  excl_scan_i64(c, kept.as<int64_t>(), koff.as<int64_t>(), items, s);
  const int64_t total = read_i64(c, koff.as<int64_t>() + items, s);
  masked_rowptr<<<gridn(m + 1), 256, 0, s>>>(ioff.as<int64_t>(), koff.as<int64_t>(), m, out->rowptr.as<int64_t>());
  SRTC_LAUNCH_CHECK("masked_rowptr");
  out->col = Buf(c, sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1), out->kind);
  out->val = Buf(c, es * (size_t)std::max<int64_t>(total, 1), out->kind);
  out->nnz = total;
  if (total > 0) {
    // item x's kept entries: from its chunk's first mask position to koff[x]
    compact_rows<V><<<gridn(items * WAVE, 256, 16384), 256, 0, s>>>(src.as<int64_t>(), koff.as<int64_t>(), items,
                                                                    colM.as<int32_t>(), valM.as<V>(),
                                                                    out->col.as<int32_t>(), out->val.as<V>());
    SRTC_LAUNCH_CHECK("compact_rows");
  }
}

void spgemm_masked(Ctx *c, int sr, int dt, IdVal id, const CsrView &A, const CsrView &B, const CsrView &M,
                   CsrOut *out, hipStream_t s) {
  if (A.n != B.m) fail(SRTC_ERR_DIM, "masked spgemm: inner dimensions differ");
  if (M.m != A.m || M.n != B.n) fail(SRTC_ERR_DIM, "masked spgemm: mask shape differs from C");
  if (B.n >= 0x7fffffff) fail(SRTC_ERR_UNSUPPORTED, "masked spgemm: more than 2^31-2 columns");
  SRTC_DISPATCH_SR(sr, dt, masked_typed, c, id, A, B, M, out, s);
}

void spgemm(Ctx *c, int sr, int dt, IdVal id, const CsrView &A, const CsrView &B, int sched, int sorted,
            CsrOut *out, SpgemmStats *st, hipStream_t s) {
  if (A.n != B.m) fail(SRTC_ERR_DIM, "spgemm: inner dimensions differ");
  if (B.n >= 0x7fffffff) fail(SRTC_ERR_UNSUPPORTED, "spgemm: more than 2^31-2 columns");
  (void)schedule(sched);
  SRTC_DISPATCH_SR(sr, dt, spgemm_typed, c, id, A, B, nullptr, sched, sorted, out, st, s);
}

void spgemm_grouped(Ctx *c, int sr, int dt, IdVal id, const CsrView &A, const CsrView &B,
                    const std::vector<RowGroup> &groups, int sorted, CsrOut *out, SpgemmStats *st, hipStream_t s) {
  if (A.n != B.m) fail(SRTC_ERR_DIM, "spgemm: inner dimensions differ");
  if (B.n >= 0x7fffffff) fail(SRTC_ERR_UNSUPPORTED, "spgemm: more than 2^31-2 columns");
  for (const RowGroup &g : groups) (void)schedule(g.sched);
  SRTC_DISPATCH_SR(sr, dt, spgemm_typed, c, id, A, B, &groups, 0, sorted, out, st, s);
}

}  // namespace srtc

namespace srtc {

// Features of an SpGEMM problem (32 scale-free numbers; the selector's
// input, Section 5.1's performance-model inputs):
//   0..9    fraction of A's rows with row length of bit length b (b >= 9 in 9)
//   10..19  fraction of rows whose product count w has (bit length + 1) / 2
//           = b (base-4 bins; bin 0 = no products, b >= 9 in 19)
//   20..23  log2 of (rows + 1), (columns of B + 1), (nnz(A) + 1), (sum w + 1)
//   24      log2 of the compression ratio: sum w / outputs over the rows
//           floor(t m / s), t < s = min(512, m) (structural outputs, counted
//           by the symbolic kernels; 1 when nothing is sampled)
//   25, 26  log2 of (max w + 1), (longest A row + 1)
//   27      coefficient of variation of w (population standard deviation /
//           mean; 0 for a zero mean)
//   28..31  the semiring, one-hot
void spgemm_features(Ctx *c, int sr, int dt, const CsrView &A, const CsrView &B, float *out, hipStream_t s) {
  for (int q = 0; q < SRTC_NUM_FEATURES; q++) out[q] = 0.f;
  const int64_t m = A.m;
  if (A.n != B.m) fail(SRTC_ERR_DIM, "features: inner dimensions differ");
  Launch L{c, s};
  Buf w(c, sizeof(int64_t) * (size_t)std::max<int64_t>(m, 1));
  if (m > 0) row_products(A, B, w.as<int64_t>(), s);
  Buf st(c, 8 * 32);
  fill_i64(st.as<int64_t>(), 32, 0, s);
  unsigned long long *hist = (unsigned long long *)st.p;
  unsigned long long *mx = hist + 21;
  double *sums = (double *)(hist + 24);
  if (m > 0) {
    feat_stats_kernel<<<gridn(m, 256, 1024), 256, 0, s>>>(A.rowptr, w.as<int64_t>(), m, hist, mx, sums);
    SRTC_LAUNCH_CHECK("feat_stats_kernel");
  }
  // sampled compression ratio
  const int64_t ns = std::min<int64_t>(512, m);
  double cr = 1.0;
  if (ns > 0 && A.nnz > 0 && B.nnz > 0) {
    std::vector<int32_t> hrows(ns);
    for (int64_t t = 0; t < ns; t++) hrows[t] = (int32_t)((t * m) / ns);
    Buf rows(c, sizeof(int32_t) * (size_t)ns), wsel(c, sizeof(int64_t) * (size_t)ns), nsel(c, sizeof(int64_t) * (size_t)ns);
    void *pin = c->host_scratch(sizeof(int32_t) * (size_t)ns);
    memcpy(pin, hrows.data(), sizeof(int32_t) * (size_t)ns);
    SRTC_HIP(hipMemcpyAsync(rows.p, pin, sizeof(int32_t) * (size_t)ns, hipMemcpyHostToDevice, s));
    gather_i64<<<gridn(ns), 256, 0, s>>>(w.as<int64_t>(), rows.as<int32_t>(), ns, wsel.as<int64_t>());
    Buf info(c, sizeof(int64_t) * INFO);
    fill_i64(info.as<int64_t>(), INFO, 0, s);
    Buf list(c, sizeof(int32_t) * (size_t)ns);
    Buf nnz_row(c, sizeof(int64_t) * (size_t)m);
    fill_i64(nnz_row.as<int64_t>(), m, 0, s);
    run_symbolic(L, schedule(0), A, B, w.as<int64_t>(), rows.as<int32_t>(), ns, info.as<int64_t>(),
                 list.as<int32_t>(), nnz_row.as<int64_t>(), info.as<int64_t>() + INFO - 1);
    gather_i64<<<gridn(ns), 256, 0, s>>>(nnz_row.as<int64_t>(), rows.as<int32_t>(), ns, nsel.as<int64_t>());
    std::vector<int64_t> hw(ns), hn(ns);
    read_to_host(c, hw.data(), wsel.p, sizeof(int64_t) * (size_t)ns, s);
    read_to_host(c, hn.data(), nsel.p, sizeof(int64_t) * (size_t)ns, s);
    double sw = 0, sn = 0;
    for (int64_t t = 0; t < ns; t++) { sw += (double)hw[t]; sn += (double)hn[t]; }
    if (sn > 0) cr = sw / sn;
  }
  uint64_t hs[32];
  read_to_host(c, hs, st.p, sizeof(hs), s);
  double dsum[2];
  memcpy(dsum, &hs[24], sizeof(dsum));
  const double mm = (double)std::max<int64_t>(m, 1);
  for (int b = 0; b < 10; b++) out[b] = (float)(hs[b] / mm);
  for (int b = 0; b < 10; b++) out[10 + b] = (float)(hs[10 + b] / mm);
  const double sw = dsum[0];
  const double mean = sw / mm;
  const double var = std::max(0.0, dsum[1] / mm - mean * mean);
  out[20] = (float)std::log2((double)m + 1);
  out[21] = (float)std::log2((double)B.n + 1);
  out[22] = (float)std::log2((double)A.nnz + 1);
  out[23] = (float)std::log2(sw + 1);
  out[24] = (float)std::log2(cr);
  out[25] = (float)std::log2((double)hs[21] + 1);
  out[26] = (float)std::log2((double)hs[22] + 1);
  out[27] = (float)(mean > 0 ? std::sqrt(var) / mean : 0.0);
  // the semiring, one-hot (the fraction of rows without products is
  // feature 10, the first bin of the product histogram)
  (void)dt;
  for (int q = 0; q < 4; q++) out[28 + q] = sr == q ? 1.f : 0.f;
}

}  // namespace srtc
