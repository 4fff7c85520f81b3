// Sparse x dense semiring products and the fixpoint steps built on them.
//
//   Y[i, c] = (+)_{k in A_i} A_ik (x) X[k, c]               (SpMM)
//   Y[i, c] = X[i, c] (+) (+)_{k in A_i} A_ik (x) X[k, c]   (Bellman-Ford step)
//
// The paper's measured kernel is exactly this sparse x dense product (MKL
// CSRMM for (+,x), a COO kernel for the tropical semiring; Section 6), and
// Bellman-Ford is P <- P (+) A (x) P on the tropical semiring (Section 4.2).
//
// Work is cut into items of at most T nonzeros of one row, so a row of any
// length costs at most T sequential gathers per lane group; G lanes (G = a
// power of two >= the dense width, up to 64) share an item, one lane per
// dense column; a wider operand is cut into chunks of 64 columns and every
// (item, chunk) pair is a unit of work of its own.  A row split into several items writes partial sums that a
// second kernel combines in item order, which keeps every semiring,
// including fp (+), deterministic.
#include <algorithm>
#include <mutex>
#include <string>

#include "internal.hpp"
#include "spmm_plan.hpp"

// The one device buffer of the product that allocates nothing: its work-item
// plan and the partial results of split rows.  Each device holds its own copy
// from the first look-up until the process ends.  Host code never passes this
// name to a kernel (on the host it is a stand-in, not a device address): it
// uses the address hipGetSymbolAddress returns for the current device.
static constexpr size_t kFixedScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace srtc {

namespace {

inline unsigned gridn(int64_t n, int bs = 256, int64_t cap = 65536) {
  int64_t g = (n + bs - 1) / bs;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

__global__ void items_count(const int64_t *rp, int64_t m, int64_t T, int64_t *cnt, int64_t *pcnt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t nz = rp[i + 1] - rp[i];
    const int64_t c = nz <= T ? 1 : (nz + T - 1) / T;
    cnt[i] = c;
    pcnt[i] = c > 1 ? c : 0;
  }
}

__global__ void items_fill(const int64_t *rp, int64_t m, int64_t T, const int64_t *ioff, const int64_t *poff,
                           int32_t *irow, int64_t *ibeg, int64_t *iend, int64_t *ipidx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = rp[i], b = rp[i + 1];
    const int64_t c = ioff[i + 1] - ioff[i];
    for (int64_t t = 0; t < c; t++) {
      const int64_t it = ioff[i] + t;
      irow[it] = (int32_t)i;
      ibeg[it] = a + t * T;
      iend[it] = std::min(b, a + (t + 1) * T);
      ipidx[it] = c > 1 ? poff[i] + t : -1;
    }
  }
}

// MODE: 0 = plain product (Y = A X, or Y (+)= A X with ACC), 1 = fixpoint
// step (self term, change flag, optional per-instance bookkeeping).
template <class SR, int G, int MODE, bool ACC>
__global__ void __launch_bounds__(256) spmm_items(const int32_t *__restrict__ irow, const int64_t *__restrict__ ibeg,
                                                  const int64_t *__restrict__ iend, const int64_t *__restrict__ ipidx,
                                                  const int64_t *__restrict__ nitems_p, const int32_t *__restrict__ cA,
                                                  const typename SR::val_t *__restrict__ vA,
                                                  const typename SR::val_t *__restrict__ X, int64_t s,
                                                  void *__restrict__ Yv, typename SR::acc_t *__restrict__ P,
                                                  typename SR::acc_t id, int32_t *changed,
                                                  const int32_t *__restrict__ row_inst,
                                                  const uint8_t *__restrict__ inst_active, int32_t *inst_changed,
                                                  const uint8_t *__restrict__ rin, uint8_t *__restrict__ rout) {
  using V = typename SR::val_t;
  using A = typename SR::acc_t;
  // (+,x) SpMM results are stored in the operand type; accumulators are A
  V *Y = reinterpret_cast<V *>(Yv);
  constexpr int PER_WAVE = WAVE / G;
  const int64_t nitems = *nitems_p;
  const int lane = lane_id();
  const int grp = lane / G, c = lane % G;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  // work units: (item, chunk of G columns); wider than G only when G = 64,
  // so each wave then takes one chunk of one item at a time
  const int64_t nch = (s + G - 1) / G;
  for (int64_t u = wave * PER_WAVE + grp; u < nitems * nch; u += nwaves * PER_WAVE) {
    const int64_t it = nch == 1 ? u : u / nch;
    const int64_t row = irow[it];
    if (MODE == 1 && row_inst && !inst_active[row_inst[row]]) continue;
    const int64_t b = ibeg[it], e = iend[it];
    const int64_t pi = ipidx[it];
    {
      const int64_t c0 = (u - it * nch) * G;
      const int64_t col = c0 + c;
      const bool on = col < s;
      A acc = id;
      if (on) {
        int64_t p = b;
        if (MODE == 1 && rin) {
          // only rows that changed in the previous step can lower this one:
          // an unchanged row's term is already part of the row's value
          for (; p + 4 <= e; p += 4) {
            const int32_t k0 = cA[p], k1 = cA[p + 1], k2 = cA[p + 2], k3 = cA[p + 3];
            const bool u0 = rin[k0], u1 = rin[k1], u2 = rin[k2], u3 = rin[k3];
            const V a0 = vA[p], a1 = vA[p + 1], a2 = vA[p + 2], a3 = vA[p + 3];
            const V x0 = u0 ? X[(int64_t)k0 * s + col] : id, x1 = u1 ? X[(int64_t)k1 * s + col] : id;
            const V x2 = u2 ? X[(int64_t)k2 * s + col] : id, x3 = u3 ? X[(int64_t)k3 * s + col] : id;
            if (!SR::absent(a0, id) && !SR::absent(x0, id)) acc = SR::add(acc, SR::mul(a0, x0));
            if (!SR::absent(a1, id) && !SR::absent(x1, id)) acc = SR::add(acc, SR::mul(a1, x1));
            if (!SR::absent(a2, id) && !SR::absent(x2, id)) acc = SR::add(acc, SR::mul(a2, x2));
            if (!SR::absent(a3, id) && !SR::absent(x3, id)) acc = SR::add(acc, SR::mul(a3, x3));
          }
          for (; p < e; p++) {
            const int32_t k = cA[p];
            if (!rin[k]) continue;
            const V a = vA[p];
            const V x = X[(int64_t)k * s + col];
            if (!SR::absent(a, id) && !SR::absent(x, id)) acc = SR::add(acc, SR::mul(a, x));
          }
        } else {
          for (; p + 4 <= e; p += 4) {
            const int32_t k0 = cA[p], k1 = cA[p + 1], k2 = cA[p + 2], k3 = cA[p + 3];
            const V a0 = vA[p], a1 = vA[p + 1], a2 = vA[p + 2], a3 = vA[p + 3];
            const V x0 = X[(int64_t)k0 * s + col], x1 = X[(int64_t)k1 * s + col];
            const V x2 = X[(int64_t)k2 * s + col], x3 = X[(int64_t)k3 * s + col];
            if (!SR::absent(a0, id) && !SR::absent(x0, id)) acc = SR::add(acc, SR::mul(a0, x0));
            if (!SR::absent(a1, id) && !SR::absent(x1, id)) acc = SR::add(acc, SR::mul(a1, x1));
            if (!SR::absent(a2, id) && !SR::absent(x2, id)) acc = SR::add(acc, SR::mul(a2, x2));
            if (!SR::absent(a3, id) && !SR::absent(x3, id)) acc = SR::add(acc, SR::mul(a3, x3));
          }
          for (; p < e; p++) {
            const int32_t k = cA[p];
            const V a = vA[p];
            const V x = X[(int64_t)k * s + col];
            if (!SR::absent(a, id) && !SR::absent(x, id)) acc = SR::add(acc, SR::mul(a, x));
          }
        }
      }
      bool diff = false;
      if (on) {
        if (pi >= 0) {
          P[pi * s + col] = acc;
        } else {
          if (MODE == 1) {
            const V old = X[row * s + col];
            if (!SR::absent(old, id)) acc = SR::add(acc, (A)old);
          }
          if (ACC) {
            const V prev = Y[row * s + col];
            if (!SR::absent(prev, id)) acc = SR::add(acc, (A)prev);
          }
          const V o = out_clamped<SR>(acc, id);
          Y[row * s + col] = o;
          if (MODE == 1) diff = o != X[row * s + col];
        }
      }
      if (MODE == 1) {
        // one store per lane group that saw a change
        const uint64_t bal = __ballot(diff);
        const uint64_t gmask = G >= WAVE ? ~0ull : (((1ull << G) - 1) << (grp * G));
        if (diff && (bal & gmask & lanemask_lt()) == 0) {
          *changed = 1;
          if (row_inst) inst_changed[row_inst[row]] = 1;
          if (rout) rout[row] = 1;
        }
      }
    }
  }
}

// Rows split into several items: combine partials in item order.
template <class SR, int G, int MODE, bool ACC>
__global__ void __launch_bounds__(256) spmm_combine(const int32_t *__restrict__ irow, const int64_t *__restrict__ ibeg,
                                                    const int64_t *__restrict__ ipidx, const int64_t *__restrict__ nitems_p,
                                                    const int64_t *__restrict__ rp, int64_t T,
                                                    const typename SR::val_t *__restrict__ X, int64_t s,
                                                    void *__restrict__ Yv, const typename SR::acc_t *__restrict__ P,
                                                    typename SR::acc_t id, int32_t *changed,
                                                    const int32_t *__restrict__ row_inst,
                                                    const uint8_t *__restrict__ inst_active, int32_t *inst_changed,
                                                    uint8_t *__restrict__ rout) {
  using V = typename SR::val_t;
  using A = typename SR::acc_t;
  V *Y = reinterpret_cast<V *>(Yv);
  constexpr int PER_WAVE = WAVE / G;
  const int64_t nitems = *nitems_p;
  const int lane = lane_id();
  const int grp = lane / G, c = lane % G;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t it = wave * PER_WAVE + grp; it < nitems; it += nwaves * PER_WAVE) {
    const int64_t pi = ipidx[it];
    const int64_t row = irow[it];
    if (pi < 0 || ibeg[it] != rp[row]) continue;  // only the first item of a split row
    if (MODE == 1 && row_inst && !inst_active[row_inst[row]]) continue;
    const int64_t nz = rp[row + 1] - rp[row];
    const int64_t cnt = (nz + T - 1) / T;
    for (int64_t c0 = 0; c0 < s; c0 += G) {
      const int64_t col = c0 + c;
      if (col >= s) continue;
      A acc = id;
      for (int64_t t = 0; t < cnt; t++) acc = SR::add(acc, P[(pi + t) * s + col]);
      if (MODE == 1) {
        const V old = X[row * s + col];
        if (!SR::absent(old, id)) acc = SR::add(acc, (A)old);
      }
      if (ACC) {
        const V prev = Y[row * s + col];
        if (!SR::absent(prev, id)) acc = SR::add(acc, (A)prev);
      }
      const V o = out_clamped<SR>(acc, id);
      Y[row * s + col] = o;
      if (MODE == 1 && o != X[row * s + col]) {
        *changed = 1;
        if (row_inst) inst_changed[row_inst[row]] = 1;
        if (rout) rout[row] = 1;
      }
    }
  }
}

template <class SR, int G, int MODE, bool ACC>
void run_items(const SpmmPlan &pl, const CsrView &A, const void *X, int64_t s, void *Y, IdVal idv,
               int32_t *changed, const int32_t *row_inst, const uint8_t *inst_active, int32_t *inst_changed,
               const uint8_t *rin, uint8_t *rout, hipStream_t st) {
  using V = typename SR::val_t;
  using Acc = typename SR::acc_t;
  const Acc id = id_as<SR>(idv);
  const int64_t nch = (s + G - 1) / G;
  const unsigned grid =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>(pl.max_items * nch * G / 256 + 1, pl.grid_cap));
  spmm_items<SR, G, MODE, ACC><<<grid, 256, 0, st>>>(pl.irow, pl.ibeg, pl.iend, pl.ipidx, pl.nitems, A.col,
                                                      (const V *)A.val, (const V *)X, s, Y, (Acc *)pl.partial, id,
                                                      changed, row_inst, inst_active, inst_changed, rin, rout);
  SRTC_LAUNCH_CHECK("spmm_items");
  if (pl.may_split) {
    spmm_combine<SR, G, MODE, ACC><<<grid, 256, 0, st>>>(pl.irow, pl.ibeg, pl.ipidx, pl.nitems, A.rowptr, pl.T,
                                                          (const V *)X, s, Y, (const Acc *)pl.partial, id, changed,
                                                          row_inst, inst_active, inst_changed, rout);
    SRTC_LAUNCH_CHECK("spmm_combine");
  }
}

template <class SR, int MODE, bool ACC>
void run_by_width(const SpmmPlan &pl, const CsrView &A, const void *X, int64_t s, void *Y, IdVal id,
                  int32_t *changed, const int32_t *row_inst, const uint8_t *inst_active, int32_t *inst_changed,
                  const uint8_t *rin, uint8_t *rout, hipStream_t st) {
  switch (pl.G) {
    case 1: run_items<SR, 1, MODE, ACC>(pl, A, X, s, Y, id, changed, row_inst, inst_active, inst_changed, rin, rout, st); break;
    case 2: run_items<SR, 2, MODE, ACC>(pl, A, X, s, Y, id, changed, row_inst, inst_active, inst_changed, rin, rout, st); break;
    case 4: run_items<SR, 4, MODE, ACC>(pl, A, X, s, Y, id, changed, row_inst, inst_active, inst_changed, rin, rout, st); break;
    case 8: run_items<SR, 8, MODE, ACC>(pl, A, X, s, Y, id, changed, row_inst, inst_active, inst_changed, rin, rout, st); break;
    case 16: run_items<SR, 16, MODE, ACC>(pl, A, X, s, Y, id, changed, row_inst, inst_active, inst_changed, rin, rout, st); break;
    case 32: run_items<SR, 32, MODE, ACC>(pl, A, X, s, Y, id, changed, row_inst, inst_active, inst_changed, rin, rout, st); break;
    default: run_items<SR, 64, MODE, ACC>(pl, A, X, s, Y, id, changed, row_inst, inst_active, inst_changed, rin, rout, st); break;
  }
}

struct SpmmCall {
  const SpmmPlan *pl;
  const CsrView *A;
  const void *X;
  int64_t s;
  void *Y;
  IdVal id;
  int mode;
  int acc;
  int32_t *changed;
  const int32_t *row_inst;
  const uint8_t *inst_active;
  int32_t *inst_changed;
  const uint8_t *rin;
  uint8_t *rout;
  hipStream_t st;
};

template <class SR> void spmm_dispatch(const SpmmCall &q) {
  if (q.mode == 1)
    run_by_width<SR, 1, false>(*q.pl, *q.A, q.X, q.s, q.Y, q.id, q.changed, q.row_inst, q.inst_active,
                               q.inst_changed, q.rin, q.rout, q.st);
  else if (q.acc)
    run_by_width<SR, 0, true>(*q.pl, *q.A, q.X, q.s, q.Y, q.id, nullptr, nullptr, nullptr, nullptr, nullptr,
                              nullptr, q.st);
  else
    run_by_width<SR, 0, false>(*q.pl, *q.A, q.X, q.s, q.Y, q.id, nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr, q.st);
}

// --------------------------------------------------------------------- BFS --
__global__ void __launch_bounds__(256) bfs_step_kernel(const int64_t *__restrict__ rp, const int32_t *__restrict__ cA,
                                                       int64_t n, const uint64_t *__restrict__ front,
                                                       uint64_t *__restrict__ visited, uint64_t *__restrict__ next,
                                                       int32_t *__restrict__ levels, int nsrc, int level,
                                                       uint64_t full, int32_t *changed) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  const int lane = lane_id();
  for (int64_t i = wid; i < n; i += nw) {
    const uint64_t vis = visited[i];
    if (vis == full) {
      if (lane == 0) next[i] = 0;
      continue;
    }
    uint64_t acc = 0;
    for (int64_t p = rp[i] + lane; p < rp[i + 1]; p += WAVE) acc |= front[cA[p]];
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) acc |= __shfl_xor(acc, d, WAVE);
    const uint64_t nw_bits = acc & ~vis & full;
    if (lane == 0) {
      next[i] = nw_bits;
      if (nw_bits) {
        visited[i] = vis | nw_bits;
        *changed = 1;
      }
    }
    if (lane < nsrc && ((nw_bits >> lane) & 1ull)) levels[i * nsrc + lane] = level;
  }
}

}  // namespace

void SpmmPlan::shape(Ctx *c, const CsrView &A, int64_t s_width) {
  ctx = c;
  rows = A.m;
  int g = 1;
  while (g < s_width && g < WAVE) g <<= 1;
  G = g;
  // a work unit is one item times one chunk of G columns: wider operands
  // have more chunks per item, so shorter items keep the units short
  T = s_width > 128 ? 64 : (G >= 64 ? 256 : (G >= 8 ? 64 : 32));
  max_items = A.m + A.nnz / T + 1;
  // a split row of z > T nonzeros has ceil(z / T) < 2 z / T items
  max_partial = 2 * (A.nnz / T) + 1;
  may_split = true;
  grid_cap = (int64_t)c->num_cus * 16;
}

void SpmmPlan::fill(const CsrView &A, int64_t *cnt_p, int64_t *pcnt_p, int64_t *ioff_p, int64_t *poff_p,
                    int64_t *sums, int32_t *irow_p, int64_t *ibeg_p, int64_t *iend_p, int64_t *ipidx_p,
                    void *partial_p, hipStream_t st) {
  const int64_t m = A.m;
  if (m > 0) {
    items_count<<<gridn(m), 256, 0, st>>>(A.rowptr, m, T, cnt_p, pcnt_p);
    SRTC_LAUNCH_CHECK("items_count");
  }
  // the two scans run one after the other on st and share the tile sums
  excl_scan_i64_ws(cnt_p, ioff_p, m, sums, st);
  excl_scan_i64_ws(pcnt_p, poff_p, m, sums, st);
  if (m > 0) {
    items_fill<<<gridn(m), 256, 0, st>>>(A.rowptr, m, T, ioff_p, poff_p, irow_p, ibeg_p, iend_p, ipidx_p);
    SRTC_LAUNCH_CHECK("items_fill");
  }
  irow = irow_p;
  ibeg = ibeg_p;
  iend = iend_p;
  ipidx = ipidx_p;
  nitems = ioff_p + m;
  partial = partial_p;
}

void SpmmPlan::build(Ctx *c, const CsrView &A, int64_t s_width, hipStream_t st) {
  shape(c, A, s_width);
  const int64_t m = A.m;
  const size_t rows = (size_t)std::max<int64_t>(m, 1);
  cnt = Buf(c, sizeof(int64_t) * rows);
  pcnt = Buf(c, sizeof(int64_t) * rows);
  ioff = Buf(c, sizeof(int64_t) * (size_t)(m + 1));
  poff = Buf(c, sizeof(int64_t) * (size_t)(m + 1));
  Buf sums(c, sizeof(int64_t) * (size_t)std::max<int64_t>(excl_scan_workspace(m), 1));
  irow_b = Buf(c, sizeof(int32_t) * (size_t)max_items);
  ibeg_b = Buf(c, sizeof(int64_t) * (size_t)max_items);
  iend_b = Buf(c, sizeof(int64_t) * (size_t)max_items);
  ipidx_b = Buf(c, sizeof(int64_t) * (size_t)max_items);
  partial_b = Buf(c, (size_t)max_partial * (size_t)s_width * 8);
  fill(A, cnt.as<int64_t>(), pcnt.as<int64_t>(), ioff.as<int64_t>(), poff.as<int64_t>(), sums.as<int64_t>(),
       irow_b.as<int32_t>(), ibeg_b.as<int64_t>(), iend_b.as<int64_t>(), ipidx_b.as<int64_t>(), partial_b.p, st);
}

namespace {
// Consecutive 256-byte aligned regions of one buffer, in the order they are
// taken; the same sequence sizes the buffer (base = null) and lays it out.
struct Carve {
  char *base;
  int64_t off = 0;
  template <class T> T *take(int64_t count) {
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += (int64_t)(((uint64_t)std::max<int64_t>(count, 1) * sizeof(T) + 255) & ~(uint64_t)255);
    return p;
  }
};

struct PlanParts {
  int64_t *cnt, *pcnt, *ioff, *poff, *sums;
  int32_t *irow;
  int64_t *ibeg, *iend, *ipidx;
  double *partial;
};

int64_t carve_plan(const SpmmPlan &pl, int64_t m, int64_t s_width, char *base, PlanParts *out) {
  Carve cv{base};
  PlanParts q;
  q.cnt = cv.take<int64_t>(m);
  q.pcnt = cv.take<int64_t>(m);
  q.ioff = cv.take<int64_t>(m + 1);
  q.poff = cv.take<int64_t>(m + 1);
  q.sums = cv.take<int64_t>(excl_scan_workspace(m));
  q.irow = cv.take<int32_t>(pl.max_items);
  q.ibeg = cv.take<int64_t>(pl.max_items);
  q.iend = cv.take<int64_t>(pl.max_items);
  q.ipidx = cv.take<int64_t>(pl.max_items);
  q.partial = cv.take<double>(pl.max_partial * s_width);
  if (out) *out = q;
  return cv.off;
}
}  // namespace

int64_t SpmmPlan::workspace_bytes(int64_t s_width) const {
  // sizes far beyond any device memory are reported as INT64_MAX instead of
  // overflowing
  const double approx = 40.0 * (double)rows + 32.0 * (double)max_items + 8.0 * (double)max_partial * (double)s_width;
  if (approx > 0x1p60) return INT64_MAX;
  return carve_plan(*this, rows, s_width, nullptr, nullptr);
}

void SpmmPlan::build_in(const CsrView &A, int64_t s_width, void *ws, hipStream_t st) {
  PlanParts q;
  carve_plan(*this, A.m, s_width, static_cast<char *>(ws), &q);
  fill(A, q.cnt, q.pcnt, q.ioff, q.poff, q.sums, q.irow, q.ibeg, q.iend, q.ipidx, q.partial, st);
}

void spmm_with_plan(const SpmmPlan &pl, int sr, int dt, IdVal id, const CsrView &A, const void *X,
                    int64_t s_width, void *Y, int mode, int accumulate, int32_t *changed, const int32_t *row_inst,
                    const uint8_t *inst_active, int32_t *inst_changed, hipStream_t st, const uint8_t *rin,
                    uint8_t *rout) {
  SpmmCall q{&pl, &A, X, s_width, Y, id, mode, accumulate, changed, row_inst, inst_active, inst_changed, rin, rout, st};
  // algorithmic bytes: A once, X once, Y written (and read for the self
  // term / accumulation)
  const double es = (double)dtype_size(dt);
  const double xy = es * (double)s_width * (double)(A.m + A.n);
  ProfScope ps(pl.ctx, mode == 1 ? "spmm.fixpoint_step" : "spmm.product",
               (4.0 + es) * A.nnz + 8.0 * (A.m + 1) + xy + (mode == 1 || accumulate ? es * s_width * A.m : 0.0), st);
  SRTC_DISPATCH_SR(sr, dt, spmm_dispatch, q);
}

void spmm(Ctx *c, int sr, int dt, IdVal id, const CsrView &A, const void *X, int64_t s_width, void *Y,
          int accumulate, hipStream_t st) {
  if (A.m == 0 || s_width == 0) return;
  SpmmPlan pl;
  pl.build(c, A, s_width, st);
  spmm_with_plan(pl, sr, dt, id, A, X, s_width, Y, 0, accumulate, nullptr, nullptr, nullptr, nullptr, st);
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void *g_fixed_ptr[kMaxDevices] = {};
}  // namespace

size_t spmm_fixed_scratch_bytes() { return kFixedScratchBytes; }

void *spmm_fixed_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) fail(SRTC_ERR_DEVICE, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_fixed_mu);
  if (!g_fixed_ptr[device]) {
    void *p = nullptr;
    SRTC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(SRTC_ERR_DEVICE, "no device address for the fixed buffer");
    g_fixed_ptr[device] = p;
  }
  return g_fixed_ptr[device];
}

void spmm_fixed(Ctx *c, int sr, int dt, IdVal id, const CsrView &A, const void *X, int64_t s_width, void *Y,
                int accumulate, hipStream_t st) {
  if (A.m == 0 || s_width == 0) return;
  if (!c->fixed_scratch) fail(SRTC_ERR_DEVICE, "the fixed buffer was not set up for this device");
  SpmmPlan pl;
  pl.shape(c, A, s_width);
  const int64_t need = pl.workspace_bytes(s_width);
  if (need > (int64_t)kFixedScratchBytes)
    fail(SRTC_ERR_TOO_LARGE, "the product's plan needs " + std::to_string(need) + " bytes; the fixed buffer holds " +
                                 std::to_string(kFixedScratchBytes) + " (call srtc_contract)");
  // every plan array is written before it is read, so the previous call's
  // contents need no clearing
  pl.build_in(A, s_width, c->fixed_scratch, st);
  // no profile record: its HIP events are resources this call must not take
  pl.ctx = nullptr;
  spmm_with_plan(pl, sr, dt, id, A, X, s_width, Y, 0, accumulate, nullptr, nullptr, nullptr, nullptr, st);
}

void bfs_step(const CsrView &A, const uint64_t *front, uint64_t *visited, uint64_t *next, int32_t *levels,
              int nsrc, int level, int32_t *changed, hipStream_t s) {
  const uint64_t full = nsrc >= 64 ? ~0ull : ((1ull << nsrc) - 1);
  bfs_step_kernel<<<gridn(A.m * WAVE, 256, 16384), 256, 0, s>>>(A.rowptr, A.col, A.m, front, visited, next,
                                                                 levels, nsrc, level, full, changed);
  SRTC_LAUNCH_CHECK("bfs_step");
}

}  // namespace srtc
