// Device primitives: exclusive scan, fills, small device->host reads.
#include "internal.hpp"

namespace srtc {

namespace {

constexpr int SCAN_BS = 256;
constexpr int SCAN_IT = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_IT;

template <class In>
__global__ void __launch_bounds__(SCAN_BS) scan_tile_sums(const In *in, int64_t n, int64_t *sums) {
  __shared__ int64_t tmp[SCAN_BS / WAVE + 1];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t acc = 0;
#pragma unroll
  for (int t = 0; t < SCAN_IT; t++) {
    int64_t i = base + (int64_t)t * SCAN_BS + threadIdx.x;
    if (i < n) acc += (int64_t)in[i];
  }
  int64_t total;
  block_excl_scan<SCAN_BS>(acc, tmp, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Scans `sums` in place (exclusive) with a single block, looping over tiles.
__global__ void __launch_bounds__(SCAN_BS) scan_sums_single(int64_t *sums, int64_t n, int64_t *total_out) {
  __shared__ int64_t tmp[SCAN_BS / WAVE + 1];
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += SCAN_TILE) {
    int64_t v[SCAN_IT];
    int64_t acc = 0;
#pragma unroll
    for (int t = 0; t < SCAN_IT; t++) {
      int64_t i = base + (int64_t)threadIdx.x * SCAN_IT + t;
      v[t] = i < n ? sums[i] : 0;
      acc += v[t];
    }
    int64_t total;
    int64_t pre = block_excl_scan<SCAN_BS>(acc, tmp, &total) + carry;
#pragma unroll
    for (int t = 0; t < SCAN_IT; t++) {
      int64_t i = base + (int64_t)threadIdx.x * SCAN_IT + t;
      if (i < n) sums[i] = pre;
      pre += v[t];
    }
    carry += total;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <class In>
__global__ void __launch_bounds__(SCAN_BS) scan_tile_down(const In *in, int64_t n, const int64_t *sums,
                                                          int64_t *out) {
  __shared__ int64_t tmp[SCAN_BS / WAVE + 1];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t v[SCAN_IT];
  int64_t acc = 0;
#pragma unroll
  for (int t = 0; t < SCAN_IT; t++) {
    int64_t i = base + (int64_t)threadIdx.x * SCAN_IT + t;
    v[t] = i < n ? (int64_t)in[i] : 0;
    acc += v[t];
  }
  int64_t total;
  int64_t pre = block_excl_scan<SCAN_BS>(acc, tmp, &total) + sums[blockIdx.x];
#pragma unroll
  for (int t = 0; t < SCAN_IT; t++) {
    int64_t i = base + (int64_t)threadIdx.x * SCAN_IT + t;
    if (i < n) out[i] = pre;
    pre += v[t];
  }
}

// The tile-sum kernel must sum the same elements the down-sweep assigns to
// a tile; both cover [base, base + SCAN_TILE), in different orders.
template <class In>
void excl_scan_into(const In *in, int64_t *out, int64_t n, int64_t *sums, hipStream_t s) {
  if (n <= 0) {
    fill_i64(out, 1, 0, s);
    return;
  }
  const int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  scan_tile_sums<In><<<(unsigned)nt, SCAN_BS, 0, s>>>(in, n, sums);
  SRTC_LAUNCH_CHECK("scan_tile_sums");
  scan_sums_single<<<1, SCAN_BS, 0, s>>>(sums, nt, out + n);
  SRTC_LAUNCH_CHECK("scan_sums_single");
  scan_tile_down<In><<<(unsigned)nt, SCAN_BS, 0, s>>>(in, n, sums, out);
  SRTC_LAUNCH_CHECK("scan_tile_down");
}

template <class In>
void excl_scan_impl(Ctx *c, const In *in, int64_t *out, int64_t n, hipStream_t s) {
  Buf sums(c, sizeof(int64_t) * (size_t)std::max<int64_t>(excl_scan_workspace(n), 1));
  excl_scan_into<In>(in, out, n, sums.as<int64_t>(), s);
}

template <class T>
__global__ void fill_kernel(T *p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <class T> void fill_any(T *p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  fill_kernel<T><<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
  SRTC_LAUNCH_CHECK("fill_kernel");
}

}  // namespace

int64_t excl_scan_workspace(int64_t n) { return n <= 0 ? 0 : (n + SCAN_TILE - 1) / SCAN_TILE; }
void excl_scan_i64(Ctx *c, const int64_t *in, int64_t *out, int64_t n, hipStream_t s) {
  excl_scan_impl<int64_t>(c, in, out, n, s);
}
void excl_scan_i64_ws(const int64_t *in, int64_t *out, int64_t n, int64_t *sums, hipStream_t s) {
  excl_scan_into<int64_t>(in, out, n, sums, s);
}
void excl_scan_i32(Ctx *c, const int32_t *in, int64_t *out, int64_t n, hipStream_t s) {
  excl_scan_impl<int32_t>(c, in, out, n, s);
}
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) { fill_any<int32_t>(p, n, v, s); }
void fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s) { fill_any<int64_t>(p, n, v, s); }

void fill_bytes_value(void *p, int64_t n, int dtype, IdVal v, hipStream_t s) {
  switch (dtype) {
    case SRTC_F64: fill_any<double>((double *)p, n, v.f, s); break;
    case SRTC_F32: fill_any<float>((float *)p, n, (float)v.f, s); break;
    case SRTC_I32: fill_any<int32_t>((int32_t *)p, n, (int32_t)v.i, s); break;
    case SRTC_BOOL8: fill_any<uint8_t>((uint8_t *)p, n, (uint8_t)v.i, s); break;
    case SRTC_BITS64: fill_any<uint64_t>((uint64_t *)p, n, (uint64_t)v.i, s); break;
    case SRTC_PATH64: fill_any<uint64_t>((uint64_t *)p, n, (uint64_t)v.i << 32, s); break;
    default: fail(SRTC_ERR_DTYPE, "fill: dtype");
  }
}

void read_to_host(Ctx *c, void *host, const void *dev, size_t bytes, hipStream_t s) {
  void *pin = c->host_scratch(bytes);
  SRTC_HIP(hipMemcpyAsync(pin, dev, bytes, hipMemcpyDeviceToHost, s));
  SRTC_HIP(hipStreamSynchronize(s));
  memcpy(host, pin, bytes);
}

int64_t read_i64(Ctx *c, const int64_t *dev, hipStream_t s) {
  int64_t v = 0;
  read_to_host(c, &v, dev, sizeof(v), s);
  return v;
}

}  // namespace srtc
