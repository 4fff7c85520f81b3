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
  void build(Ctx *c, const CsrView &A, int64_t s_width, hipStream_t st);
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

}  // namespace srtc
