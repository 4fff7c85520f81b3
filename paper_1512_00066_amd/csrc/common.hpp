// Shared definitions for the srtc HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/srtc.h"

namespace srtc {

// ----------------------------------------------------------------- errors --
// Internal failures are C++ exceptions; every C-ABI entry point catches them
// and turns them into a status plus a message.
struct Error {
  srtc_status st;
  std::string msg;
};

[[noreturn]] inline void fail(srtc_status st, const std::string &msg) { throw Error{st, msg}; }

inline void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) fail(SRTC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define SRTC_HIP(x) ::srtc::hip_check((x), #x)
#define SRTC_LAUNCH_CHECK(name) ::srtc::hip_check(hipGetLastError(), name)

// ---------------------------------------------------------------- context --
struct Ctx;

// Device buffer from the context allocator, returned on scope exit.
// kind SCRATCH: stream-ordered pool memory released when the call ends;
// kind OUTPUT: the caller's allocator (the buffer is handed over).
enum BufKind { SCRATCH = 0, OUTPUT = 1 };
struct Buf {
  Ctx *ctx = nullptr;
  void *p = nullptr;
  size_t bytes = 0;
  int kind = SCRATCH;
  Buf() = default;
  Buf(Ctx *c, size_t n, int k = SCRATCH);
  Buf(const Buf &) = delete;
  Buf &operator=(const Buf &) = delete;
  Buf(Buf &&o) noexcept : ctx(o.ctx), p(o.p), bytes(o.bytes), kind(o.kind) { o.p = nullptr; }
  Buf &operator=(Buf &&o) noexcept;
  ~Buf();
  template <class T> T *as() const { return reinterpret_cast<T *>(p); }
  void *release() { void *q = p; p = nullptr; return q; }
};

// ------------------------------------------------------------ wave helpers --
constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// DPP lane moves (GFX9 data-parallel primitives): lanes whose source is
// outside the pattern, or whose row is masked off, read 0.  Values of 8 bytes
// move as two 32-bit halves.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWMASK, 0xf, false);
}
template <int CTRL, int ROWMASK, class T>
__device__ __forceinline__ T dpp_move(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "dpp_move on 4- or 8-byte values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp32<CTRL, ROWMASK>(__builtin_bit_cast(uint32_t, v)));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint64_t hi = dpp32<CTRL, ROWMASK>((uint32_t)(u >> 32));
    const uint64_t lo = dpp32<CTRL, ROWMASK>((uint32_t)u);
    return __builtin_bit_cast(T, (hi << 32) | lo);
  }
}

// Inclusive sum over the 64 lanes: shifts of 1, 2, 4, 8 within each row of
// 16 lanes, then lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31
// into rows 2 and 3.
template <class T> __device__ __forceinline__ T wave_incl_scan(T v) {
  v += dpp_move<0x111, 0xf>(v);  // row_shr:1
  v += dpp_move<0x112, 0xf>(v);  // row_shr:2
  v += dpp_move<0x114, 0xf>(v);  // row_shr:4
  v += dpp_move<0x118, 0xf>(v);  // row_shr:8
  v += dpp_move<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_move<0x143, 0xc>(v);  // row_bcast:31
  return v;
}

template <class T> __device__ __forceinline__ T lane63(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    return __builtin_bit_cast(T, (hi << 32) | lo);
  }
}

// Sum over the 64 lanes (every lane gets it); all lanes must be active.
template <class T> __device__ __forceinline__ T wave_sum(T v) { return lane63(wave_incl_scan(v)); }

// Block-wide exclusive scan for BS threads (BS a multiple of 64, <= 1024).
// `tmp` is LDS of at least BS/64 + 1 elements.  Returns the exclusive prefix
// and writes the block total to *total (every thread sees it).  With
// SYNC_AFTER false the caller must pass a barrier before tmp is written
// again (by any later scan on the same tmp).
template <int BS, class T, bool SYNC_AFTER = true>
__device__ __forceinline__ T block_excl_scan(T v, T *tmp, T *total) {
  static_assert(BS % WAVE == 0 && BS <= 1024, "block size");
  constexpr int NW = BS / WAVE;
  const int w = threadIdx.x / WAVE;
  const T inc = wave_incl_scan(v);
  if (lane_id() == WAVE - 1) tmp[w] = inc;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < NW; q++) {
    const T x = tmp[q];
    if (q < w) before += x;
    tot += x;
  }
  *total = tot;
  if (SYNC_AFTER) __syncthreads();
  return before + inc - v;
}

// ------------------------------------------------------------- semirings --
// Semirings as compile-time functors (Section 3.1 of the paper: additive op
// with its identity, multiplicative op).  The identity itself is a runtime
// value (the caller's add_id) held as acc_t.
//   val_t   stored element type
//   acc_t   accumulator type (LDS / registers)
//   mul     product of two present entries, as acc_t
//   add     additive op on accumulators
//   lds_add atomic additive op on an LDS accumulator
//   absent  whether a stored value equals the identity
//   out     accumulator -> stored value
// (+,x) on fp32 forms the exact product in fp64 and accumulates in fp64.

template <class T> struct PlusTimes {
  using val_t = T;
  using acc_t = double;
  static constexpr int SR = SRTC_PLUS_TIMES;
  static constexpr bool HAS_VALS = true;
  __device__ static acc_t mul(val_t a, val_t b) { return (acc_t)a * (acc_t)b; }
  __device__ static acc_t add(acc_t a, acc_t b) { return a + b; }
  __device__ static void lds_add(acc_t *p, acc_t v) { atomicAdd(p, v); }
  __device__ static bool absent(val_t v, acc_t id) { return (acc_t)v == id; }
  __device__ static bool acc_absent(acc_t v, acc_t id) { return v == id; }
  __device__ static val_t out(acc_t v) { return (val_t)v; }
};

template <class T> struct MinPlus;
template <> struct MinPlus<int32_t> {
  using val_t = int32_t;
  using acc_t = int32_t;
  static constexpr int SR = SRTC_MIN_PLUS;
  static constexpr bool HAS_VALS = true;
  __device__ static acc_t mul(val_t a, val_t b) { return a + b; }
  __device__ static acc_t add(acc_t a, acc_t b) { return a < b ? a : b; }
  __device__ static void lds_add(acc_t *p, acc_t v) { atomicMin(p, v); }
  __device__ static bool absent(val_t v, acc_t id) { return v == id; }
  // accumulators start at id and only decrease, so ">= id" is "== id"
  __device__ static bool acc_absent(acc_t v, acc_t id) { return v >= id; }
  __device__ static val_t out(acc_t v) { return v; }
};
template <> struct MinPlus<float> {
  using val_t = float;
  using acc_t = float;
  static constexpr int SR = SRTC_MIN_PLUS;
  static constexpr bool HAS_VALS = true;
  __device__ static acc_t mul(val_t a, val_t b) { return a + b; }
  __device__ static acc_t add(acc_t a, acc_t b) { return a < b ? a : b; }
  __device__ static void lds_add(acc_t *p, acc_t v) { atomicMin(p, v); }
  __device__ static bool absent(val_t v, acc_t id) { return v == id; }
  __device__ static bool acc_absent(acc_t v, acc_t id) { return v >= id; }
  __device__ static val_t out(acc_t v) { return v; }
};

struct OrAnd {
  using val_t = uint8_t;
  using acc_t = uint32_t;
  static constexpr int SR = SRTC_OR_AND;
  static constexpr bool HAS_VALS = false;  // present entries are all "true"
  __device__ static acc_t mul(val_t, val_t) { return 1u; }
  __device__ static acc_t add(acc_t a, acc_t b) { return a | b; }
  __device__ static void lds_add(acc_t *p, acc_t v) { *p = v; }
  __device__ static bool absent(val_t v, acc_t) { return v == 0; }
  __device__ static bool acc_absent(acc_t v, acc_t) { return v == 0; }
  __device__ static val_t out(acc_t v) { return (val_t)(v != 0); }
};

// (min,+) on paths packed as (weight << 32) | hops: the unsigned minimum is
// the lexicographic one (lighter path first, fewer hops on a tie) and the
// product adds weights and hops without a carry between the halves.  A
// weight at or above the identity's is the absent path.
struct MinPlusPath {
  using val_t = uint64_t;
  using acc_t = uint64_t;
  static constexpr int SR = SRTC_MIN_PLUS;
  static constexpr bool HAS_VALS = true;
  __device__ static acc_t mul(val_t a, val_t b) { return a + b; }
  __device__ static acc_t add(acc_t a, acc_t b) { return a < b ? a : b; }
  __device__ static void lds_add(acc_t *p, acc_t v) { atomicMin((unsigned long long *)p, (unsigned long long)v); }
  __device__ static bool absent(val_t v, acc_t id) { return (v >> 32) >= (id >> 32); }
  __device__ static bool acc_absent(acc_t v, acc_t id) { return (v >> 32) >= (id >> 32); }
  __device__ static val_t out(acc_t v) { return v; }
};

template <class T> struct MaxTimes {
  using val_t = T;
  using acc_t = T;
  static constexpr int SR = SRTC_MAX_TIMES;
  static constexpr bool HAS_VALS = true;
  __device__ static acc_t mul(val_t a, val_t b) { return a * b; }
  __device__ static acc_t add(acc_t a, acc_t b) { return a > b ? a : b; }
  __device__ static void lds_add(acc_t *p, acc_t v) { atomicMax(p, v); }
  __device__ static bool absent(val_t v, acc_t id) { return v == id; }
  __device__ static bool acc_absent(acc_t v, acc_t id) { return v <= id; }
  __device__ static val_t out(acc_t v) { return v; }
};

// The stored form of an accumulator in a dense output: a result that counts
// as absent (for (min,+) int32 a sum at or above the identity, Section 3.1's
// reading that such sums are no path) is written as the identity itself, so
// a dense result never holds a value beyond it.
template <class SR>
__device__ __forceinline__ typename SR::val_t out_clamped(typename SR::acc_t v, typename SR::acc_t id) {
  return SR::acc_absent(v, id) ? SR::out(id) : SR::out(v);
}

// Identity holder passed to kernels: the caller's add_id converted once.
struct IdVal {
  double f;
  int64_t i;
};

template <class SR> inline typename SR::acc_t id_as(const IdVal &v);
template <> inline double id_as<PlusTimes<double>>(const IdVal &v) { return v.f; }
template <> inline double id_as<PlusTimes<float>>(const IdVal &v) { return v.f; }
template <> inline int32_t id_as<MinPlus<int32_t>>(const IdVal &v) { return (int32_t)v.i; }
template <> inline float id_as<MinPlus<float>>(const IdVal &v) { return (float)v.f; }
template <> inline uint32_t id_as<OrAnd>(const IdVal &) { return 0u; }
template <> inline float id_as<MaxTimes<float>>(const IdVal &v) { return (float)v.f; }
template <> inline double id_as<MaxTimes<double>>(const IdVal &v) { return v.f; }
template <> inline uint64_t id_as<MinPlusPath>(const IdVal &v) { return (uint64_t)v.i << 32; }

// Dispatch a functor template over the (semiring, dtype) pairs.
#define SRTC_DISPATCH_SR(sr, dt, F, ...)                                                 \
  do {                                                                                   \
    if ((sr) == SRTC_PLUS_TIMES && (dt) == SRTC_F64) F<::srtc::PlusTimes<double>>(__VA_ARGS__); \
    else if ((sr) == SRTC_PLUS_TIMES && (dt) == SRTC_F32) F<::srtc::PlusTimes<float>>(__VA_ARGS__); \
    else if ((sr) == SRTC_MIN_PLUS && (dt) == SRTC_I32) F<::srtc::MinPlus<int32_t>>(__VA_ARGS__); \
    else if ((sr) == SRTC_MIN_PLUS && (dt) == SRTC_F32) F<::srtc::MinPlus<float>>(__VA_ARGS__); \
    else if ((sr) == SRTC_MIN_PLUS && (dt) == SRTC_PATH64) F<::srtc::MinPlusPath>(__VA_ARGS__); \
    else if ((sr) == SRTC_OR_AND && (dt) == SRTC_BOOL8) F<::srtc::OrAnd>(__VA_ARGS__);      \
    else if ((sr) == SRTC_MAX_TIMES && (dt) == SRTC_F32) F<::srtc::MaxTimes<float>>(__VA_ARGS__); \
    else if ((sr) == SRTC_MAX_TIMES && (dt) == SRTC_F64) F<::srtc::MaxTimes<double>>(__VA_ARGS__); \
    else ::srtc::fail(SRTC_ERR_DTYPE, "value type not defined for this semiring");        \
  } while (0)

inline size_t dtype_size(int dt) {
  switch (dt) {
    case SRTC_F64: return 8;
    case SRTC_F32: return 4;
    case SRTC_I32: return 4;
    case SRTC_BOOL8: return 1;
    case SRTC_BITS64: return 8;
    case SRTC_PATH64: return 8;
  }
  fail(SRTC_ERR_DTYPE, "unknown dtype");
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace srtc
