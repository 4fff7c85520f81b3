// Fold: index-value pairs -> CSR matrix (the mode folding of Section 5.1 and
// the local transposition/reordering of Section 6.2).
//
// Keys (row*ncols + col) are sorted by a stable LSD radix sort whose per-tile
// digit ranking runs in LDS with wave ballots; equal keys then form segments
// that are combined with the semiring's additive op in input order (float (+)
// accumulated in fp64 and rounded once), identity results are dropped and
// the row pointer is filled from the row boundaries of the sorted output.
#include "internal.hpp"

namespace srtc {

namespace {

constexpr int RS_BS = 256;            // threads per tile
constexpr int RS_IT = 8;              // keys per thread
constexpr int RS_TILE = RS_BS * RS_IT;
constexpr int RS_NW = RS_BS / WAVE;
constexpr int RS_DIG = 256;           // 8-bit digits

__global__ void __launch_bounds__(RS_BS) radix_hist(const uint64_t *keys, int64_t n, int shift,
                                                    int32_t *hist, int64_t ntiles) {
  __shared__ int32_t cnt[RS_DIG];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll
  for (int r = 0; r < RS_IT; r++) {
    int64_t i = base + (int64_t)r * RS_BS + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xFF], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one tile.  Items are visited round by round (item r of
// thread t is tile position r*RS_BS + t), so tile order is round-major, then
// wave, then lane; ranks follow that order.
__global__ void __launch_bounds__(RS_BS) radix_scatter(const uint64_t *kin, const uint32_t *pin,
                                                       uint64_t *kout, uint32_t *pout, int64_t n,
                                                       int shift, const int64_t *offs,
                                                       int64_t ntiles) {
  __shared__ int32_t wcnt[RS_NW][RS_DIG];
  __shared__ int32_t run[RS_DIG];
  __shared__ int32_t tstart[RS_DIG];
  __shared__ int32_t scan_tmp[RS_NW + 1];
  __shared__ uint64_t skey[RS_TILE];
  __shared__ uint32_t spay[RS_TILE];

  const int t = threadIdx.x;
  const int w = t / WAVE;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  run[t] = 0;
#pragma unroll
  for (int q = 0; q < RS_NW; q++) wcnt[q][t] = 0;
  __syncthreads();

  uint64_t key[RS_IT];
  uint32_t pay[RS_IT];
  int32_t rank[RS_IT];
  int dig[RS_IT];
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < RS_IT; r++) {
    const int64_t i = base + (int64_t)r * RS_BS + t;
    const bool valid = i < n;
    key[r] = valid ? kin[i] : 0;
    pay[r] = valid ? pin[i] : 0;
    const int d = (int)((key[r] >> shift) & 0xFF);
    dig[r] = d;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const uint64_t m = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? m : ~m;
    }
    int rw = __popcll(peers & lt);
    if (valid && rw == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pre = run[d];
      for (int q = 0; q < w; q++) pre += wcnt[q][d];
      rank[r] = pre + rw;
    } else {
      rank[r] = -1;
    }
    __syncthreads();
    {
      int add = 0;
#pragma unroll
      for (int q = 0; q < RS_NW; q++) { add += wcnt[q][t]; wcnt[q][t] = 0; }
      run[t] += add;
    }
    __syncthreads();
  }
  // tile-local start of each digit
  int32_t total;
  int32_t st = block_excl_scan<RS_BS>(run[t], scan_tmp, &total);
  tstart[t] = st;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RS_IT; r++) {
    if (rank[r] >= 0) {
      const int p = tstart[dig[r]] + rank[r];
      skey[p] = key[r];
      spay[p] = pay[r];
    }
  }
  __syncthreads();
  for (int p = t; p < total; p += RS_BS) {
    const uint64_t k = skey[p];
    const int d = (int)((k >> shift) & 0xFF);
    const int64_t dst = offs[(int64_t)d * ntiles + blockIdx.x] + (p - tstart[d]);
    kout[dst] = k;
    pout[dst] = spay[p];
  }
}

__global__ void iota_u32(uint32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (uint32_t)i;
}

__global__ void seg_heads(const int64_t *keys, int64_t n, int32_t *flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// starts[segid] = first position of each segment; starts[nseg] = n.
__global__ void seg_starts(const int32_t *flag, const int64_t *segid, int64_t n, int64_t *starts) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (flag[i]) starts[segid[i]] = i;
    if (i == n - 1) starts[segid[n]] = n;
  }
}

// One thread per segment: combine its values in sorted (= input) order.
template <class SR>
__global__ void seg_reduce(const int64_t *keys, const uint32_t *perm, const void *vals_in,
                           const int64_t *starts, const int64_t *nseg_p, int64_t n,
                           typename SR::acc_t id, int32_t *keep, typename SR::val_t *sval) {
  using V = typename SR::val_t;
  using A = typename SR::acc_t;
  const V *vals = reinterpret_cast<const V *>(vals_in);
  const int64_t nseg = *nseg_p;
  for (int64_t sgi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sgi < n;
       sgi += (int64_t)gridDim.x * blockDim.x) {
    if (sgi >= nseg) { keep[sgi] = 0; continue; }
    const int64_t a = starts[sgi], b = starts[sgi + 1];
    A acc = id;
    bool any = false;
    for (int64_t j = a; j < b; j++) {
      const V v = vals[perm[j]];
      if (SR::absent(v, id)) continue;
      const A x = SR::HAS_VALS ? (A)v : (A)1;
      acc = any ? SR::add(acc, x) : x;
      any = true;
    }
    const V o = SR::out(acc);
    const bool k = any && !SR::absent(o, id);
    keep[sgi] = k ? 1 : 0;
    sval[sgi] = o;
  }
}

template <class V>
__global__ void seg_write(const int64_t *keys, const int64_t *starts, const int32_t *keep,
                          const int64_t *pos, const V *sval, const int64_t *nseg_p, int64_t ncols,
                          int32_t *col, V *val, int64_t *orow) {
  const int64_t nseg = *nseg_p;
  for (int64_t sgi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sgi < nseg;
       sgi += (int64_t)gridDim.x * blockDim.x) {
    if (!keep[sgi]) continue;
    const int64_t k = keys[starts[sgi]];
    const int64_t o = pos[sgi];
    col[o] = (int32_t)(k % ncols);
    val[o] = sval[sgi];
    orow[o] = k / ncols;
  }
}

// rowptr from the (sorted) row of every output entry; each rowptr slot is
// written exactly once.
__global__ void rowptr_from_rows(const int64_t *orow, int64_t nnz, int64_t nrows, int64_t *rowptr) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (nnz == 0) {
    for (int64_t r = gid; r <= nrows; r += stride) rowptr[r] = 0;
    return;
  }
  for (int64_t p = gid; p < nnz; p += stride) {
    const int64_t r = orow[p];
    if (p == 0)
      for (int64_t q = 0; q <= r; q++) rowptr[q] = 0;
    else {
      const int64_t r0 = orow[p - 1];
      for (int64_t q = r0 + 1; q <= r; q++) rowptr[q] = p;
    }
    if (p == nnz - 1)
      for (int64_t q = r + 1; q <= nrows; q++) rowptr[q] = nnz;
  }
}

struct RemapArgs {
  int64_t dims[SRTC_MAX_ORDER];
  int order;
  int nr, nc;
  int rmode[SRTC_MAX_ORDER];
  int cmode[SRTC_MAX_ORDER];
  int64_t ncols;
};

__global__ void remap_kernel(const int64_t *keys, int64_t n, RemapArgs a, int64_t *out) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t idx[SRTC_MAX_ORDER];
    int64_t k = keys[t];
    for (int m = a.order - 1; m >= 0; m--) {
      idx[m] = k % a.dims[m];
      k /= a.dims[m];
    }
    int64_t r = 0, c = 0;
    for (int q = 0; q < a.nr; q++) r = r * a.dims[a.rmode[q]] + idx[a.rmode[q]];
    for (int q = 0; q < a.nc; q++) c = c * a.dims[a.cmode[q]] + idx[a.cmode[q]];
    out[t] = r * a.ncols + c;
  }
}

__global__ void csr_keys_kernel(const int64_t *rowptr, const int32_t *col, int64_t m, int64_t ncols,
                                int64_t *keys) {
  // one wave per row
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  for (int64_t i = wid; i < m; i += nw)
    for (int64_t p = rowptr[i] + lane_id(); p < rowptr[i + 1]; p += WAVE) keys[p] = i * ncols + col[p];
}

inline unsigned grid_for(int64_t n, int bs = 256, int64_t cap = 65536) {
  int64_t g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

template <class SR>
void seg_reduce_launch(const int64_t *keys, const uint32_t *perm, const void *vals,
                       const int64_t *starts, const int64_t *nseg, int64_t n, IdVal id,
                       int32_t *keep, void *sval, hipStream_t s) {
  seg_reduce<SR><<<grid_for(n), 256, 0, s>>>(keys, perm, vals, starts, nseg, n, id_as<SR>(id), keep,
                                             reinterpret_cast<typename SR::val_t *>(sval));
  SRTC_LAUNCH_CHECK("seg_reduce");
}

template <class V>
void seg_write_launch(const int64_t *keys, const int64_t *starts, const int32_t *keep,
                      const int64_t *pos, const void *sval, const int64_t *nseg, int64_t n,
                      int64_t ncols, int32_t *col, void *val, int64_t *orow, hipStream_t s) {
  seg_write<V><<<grid_for(n), 256, 0, s>>>(keys, starts, keep, pos, (const V *)sval, nseg, ncols, col,
                                           (V *)val, orow);
  SRTC_LAUNCH_CHECK("seg_write");
}

}  // namespace

void radix_sort_pairs(Ctx *c, int64_t *keys, uint32_t *payload, int64_t n, int bits,
                      hipStream_t s) {
  if (n <= 1 || bits <= 0) return;
  const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
  Buf k2(c, sizeof(uint64_t) * (size_t)n), p2(c, sizeof(uint32_t) * (size_t)n);
  Buf hist(c, sizeof(int32_t) * (size_t)(RS_DIG * ntiles));
  Buf offs(c, sizeof(int64_t) * (size_t)(RS_DIG * ntiles + 1));
  uint64_t *ka = reinterpret_cast<uint64_t *>(keys), *kb = k2.as<uint64_t>();
  uint32_t *pa = payload, *pb = p2.as<uint32_t>();
  const int passes = (bits + 7) / 8;
  for (int ps = 0; ps < passes; ps++) {
    const int shift = ps * 8;
    {
      ProfScope ps(c, "fold.radix_hist", 8.0 * n + 4.0 * RS_DIG * ntiles, s);
      radix_hist<<<(unsigned)ntiles, RS_BS, 0, s>>>(ka, n, shift, hist.as<int32_t>(), ntiles);
      SRTC_LAUNCH_CHECK("radix_hist");
    }
    excl_scan_i32(c, hist.as<int32_t>(), offs.as<int64_t>(), RS_DIG * ntiles, s);
    {
      ProfScope ps(c, "fold.radix_scatter", 24.0 * n + 8.0 * RS_DIG * ntiles, s);
      radix_scatter<<<(unsigned)ntiles, RS_BS, 0, s>>>(ka, pa, kb, pb, n, shift, offs.as<int64_t>(), ntiles);
      SRTC_LAUNCH_CHECK("radix_scatter");
    }
    std::swap(ka, kb);
    std::swap(pa, pb);
  }
  if (ka != reinterpret_cast<uint64_t *>(keys)) {
    SRTC_HIP(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    SRTC_HIP(hipMemcpyAsync(payload, pa, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
  }
}

void fold_keys_to_csr(Ctx *c, int sr, int dt, IdVal id, const int64_t *keys_in, const void *vals,
                      int64_t nnz, int64_t nrows, int64_t ncols, CsrOut *out, hipStream_t s) {
  if (nnz >= (int64_t(1) << 32)) fail(SRTC_ERR_UNSUPPORTED, "fold: more than 2^32 entries");
  const size_t es = dtype_size(dt);
  out->m = nrows;
  out->n = ncols;
  out->rowptr = Buf(c, sizeof(int64_t) * (size_t)(nrows + 1), out->kind);
  if (nnz == 0) {
    fill_i64(out->rowptr.as<int64_t>(), nrows + 1, 0, s);
    out->nnz = 0;
    out->col = Buf(c, 4, out->kind);
    out->val = Buf(c, es, out->kind);
    return;
  }
  // sort (key, original position)
  Buf keys(c, sizeof(int64_t) * (size_t)nnz), perm(c, sizeof(uint32_t) * (size_t)nnz);
  SRTC_HIP(hipMemcpyAsync(keys.p, keys_in, sizeof(int64_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
  iota_u32<<<grid_for(nnz), 256, 0, s>>>(perm.as<uint32_t>(), nnz);
  SRTC_LAUNCH_CHECK("iota_u32");
  const unsigned __int128 span = (unsigned __int128)nrows * (unsigned __int128)ncols;
  int bits = 0;
  while (bits < 63 && ((unsigned __int128)1 << bits) < span) bits++;
  c->tracef("fold: %lld keys, %lld x %lld, %d key bits", (long long)nnz, (long long)nrows, (long long)ncols, bits);
  radix_sort_pairs(c, keys.as<int64_t>(), perm.as<uint32_t>(), nnz, bits, s);
  // segments of equal keys
  Buf flag(c, sizeof(int32_t) * (size_t)nnz), segid(c, sizeof(int64_t) * (size_t)(nnz + 1));
  seg_heads<<<grid_for(nnz), 256, 0, s>>>(keys.as<int64_t>(), nnz, flag.as<int32_t>());
  SRTC_LAUNCH_CHECK("seg_heads");
  excl_scan_i32(c, flag.as<int32_t>(), segid.as<int64_t>(), nnz, s);
  Buf starts(c, sizeof(int64_t) * (size_t)(nnz + 1));
  seg_starts<<<grid_for(nnz), 256, 0, s>>>(flag.as<int32_t>(), segid.as<int64_t>(), nnz,
                                           starts.as<int64_t>());
  SRTC_LAUNCH_CHECK("seg_starts");
  const int64_t *nseg = segid.as<int64_t>() + nnz;
  Buf keep(c, sizeof(int32_t) * (size_t)nnz), sval(c, es * (size_t)nnz);
  SRTC_DISPATCH_SR(sr, dt, seg_reduce_launch, keys.as<int64_t>(), perm.as<uint32_t>(), vals,
                   starts.as<int64_t>(), nseg, nnz, id, keep.as<int32_t>(), sval.p, s);
  Buf pos(c, sizeof(int64_t) * (size_t)(nnz + 1));
  excl_scan_i32(c, keep.as<int32_t>(), pos.as<int64_t>(), nnz, s);
  const int64_t total = read_i64(c, pos.as<int64_t>() + nnz, s);
  c->tracef("fold: %lld entries after combining duplicates", (long long)total);
  out->nnz = total;
  out->col = Buf(c, sizeof(int32_t) * (size_t)(total > 0 ? total : 1), out->kind);
  out->val = Buf(c, es * (size_t)(total > 0 ? total : 1), out->kind);
  Buf orow(c, sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
  switch (es) {
    case 8: seg_write_launch<uint64_t>(keys.as<int64_t>(), starts.as<int64_t>(), keep.as<int32_t>(),
                                       pos.as<int64_t>(), sval.p, nseg, nnz, ncols, out->col.as<int32_t>(),
                                       out->val.p, orow.as<int64_t>(), s); break;
    case 4: seg_write_launch<uint32_t>(keys.as<int64_t>(), starts.as<int64_t>(), keep.as<int32_t>(),
                                       pos.as<int64_t>(), sval.p, nseg, nnz, ncols, out->col.as<int32_t>(),
                                       out->val.p, orow.as<int64_t>(), s); break;
    default: seg_write_launch<uint8_t>(keys.as<int64_t>(), starts.as<int64_t>(), keep.as<int32_t>(),
                                       pos.as<int64_t>(), sval.p, nseg, nnz, ncols, out->col.as<int32_t>(),
                                       out->val.p, orow.as<int64_t>(), s); break;
  }
  rowptr_from_rows<<<grid_for(total > 0 ? total : nrows + 1), 256, 0, s>>>(orow.as<int64_t>(), total, nrows,
                                                                          out->rowptr.as<int64_t>());
  SRTC_LAUNCH_CHECK("rowptr_from_rows");
}

void remap_keys(Ctx *, const int64_t *keys, int64_t nnz, int order, const int64_t *dims,
                int nrow_modes, const int *row_modes, int ncol_modes, const int *col_modes,
                int64_t *out, hipStream_t s) {
  if (nnz == 0) return;
  RemapArgs a{};
  a.order = order;
  for (int m = 0; m < order; m++) a.dims[m] = dims[m];
  a.nr = nrow_modes;
  a.nc = ncol_modes;
  a.ncols = 1;
  for (int q = 0; q < nrow_modes; q++) a.rmode[q] = row_modes[q];
  for (int q = 0; q < ncol_modes; q++) { a.cmode[q] = col_modes[q]; a.ncols *= dims[col_modes[q]]; }
  remap_kernel<<<grid_for(nnz), 256, 0, s>>>(keys, nnz, a, out);
  SRTC_LAUNCH_CHECK("remap_kernel");
}

void csr_to_keys(const CsrView &a, int64_t *keys, hipStream_t s) {
  if (a.nnz == 0 || a.m == 0) return;
  csr_keys_kernel<<<grid_for(a.m * WAVE, 256, 16384), 256, 0, s>>>(a.rowptr, a.col, a.m, a.n, keys);
  SRTC_LAUNCH_CHECK("csr_keys_kernel");
}

}  // namespace srtc
