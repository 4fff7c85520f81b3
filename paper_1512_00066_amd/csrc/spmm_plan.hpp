// Work items of a sparse x dense product (rows cut into pieces of at most T
// nonzeros); built once per matrix and reused by every fixpoint step.
#pragma once

#include "internal.hpp"

namespace srtc {

struct SpmmPlan {
  Ctx *ctx = nullptr;
  int G = 64;          // lanes per item (power of two covering the width)
  int64_t T = 256;     // nonzeros per item
  int64_t max_items = 0;
  int64_t grid_cap = 4096;
  bool may_split = true;
  Buf cnt, pcnt, ioff, poff, irow_b, ibeg_b, iend_b, ipidx_b, partial_b;
  const int32_t *irow = nullptr;
  const int64_t *ibeg = nullptr, *iend = nullptr, *ipidx = nullptr, *nitems = nullptr;
  void *partial = nullptr;
  int64_t rows = 0;         // rows of A
  int64_t max_partial = 0;  // rows of s_width accumulators for split rows
  // item length, lanes per item and buffer sizes for A and s_width
  void shape(Ctx *c, const CsrView &A, int64_t s_width);
  // shape, then allocate the buffers from the context and fill them
  void build(Ctx *c, const CsrView &A, int64_t s_width, hipStream_t st);
  // bytes of one caller-supplied buffer holding every plan array
  int64_t workspace_bytes(int64_t s_width) const;
  // shape() first; lays the plan out in ws (workspace_bytes, 256-byte
  // aligned) and fills it; allocates nothing
  void build_in(const CsrView &A, int64_t s_width, void *ws, hipStream_t st);

 private:
  void fill(const CsrView &A, int64_t *cnt_p, int64_t *pcnt_p, int64_t *ioff_p, int64_t *poff_p, int64_t *sums,
            int32_t *irow_p, int64_t *ibeg_p, int64_t *iend_p, int64_t *ipidx_p, void *partial_p, hipStream_t st);
};

// mode 0: Y = A (x) X (accumulate: Y (+)= A (x) X); mode 1: fixpoint step
// Y = X (+) A (x) X raising *changed (and per-instance flags) on change.
// In mode 1, rin (one byte per row, optional) limits the gathers to rows
// that changed in the previous step, and rout (optional) marks the rows
// this step changed; both need an idempotent additive op.
void spmm_with_plan(const SpmmPlan &pl, int sr, int dt, IdVal id, const CsrView &A, const void *X,
                    int64_t s_width, void *Y, int mode, int accumulate, int32_t *changed, const int32_t *row_inst,
                    const uint8_t *inst_active, int32_t *inst_changed, hipStream_t st, const uint8_t *rin = nullptr,
                    uint8_t *rout = nullptr);

// The sparse x dense product with its plan in the library's fixed per-device
// buffer: Y = A (x) X (accumulate: Y (+)= A (x) X).  No device memory is
// allocated; SRTC_ERR_TOO_LARGE if the plan needs more than
// spmm_fixed_scratch_bytes().  Calls that overlap on one device race.
void spmm_fixed(Ctx *c, int sr, int dt, IdVal id, const CsrView &A, const void *X, int64_t s_width, void *Y,
                int accumulate, hipStream_t st);
size_t spmm_fixed_scratch_bytes();
// Device address of the fixed buffer on `device` (the current device),
// looked up once per device and kept for the life of the process.
void *spmm_fixed_scratch_init(int device);

}  // namespace srtc
