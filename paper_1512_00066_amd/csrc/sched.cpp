// Scheduling entry points: features, exhaustive autotuning.
//
// The paper tunes over a space of decompositions with cost models (Section
// 5.1) and reports the median of ten runs after one warm-up (Section 6);
// here the space is the SpGEMM schedule table and the cost is measured.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

using namespace srtc;

namespace {

CsrView matrix_view(const srtc_tensor *t, const char *name) {
  if (!t) fail(SRTC_ERR_ARG, std::string(name) + ": null");
  if (t->format != SRTC_CSR || t->order != 2 || t->split != 1)
    fail(SRTC_ERR_FORMAT, std::string(name) + ": a CSR matrix (order 2, split 1) is required");
  CsrView v;
  v.m = t->dims[0];
  v.n = t->dims[1];
  v.nnz = t->nnz;
  v.rowptr = t->rowptr;
  v.col = t->colidx;
  v.val = t->vals;
  return v;
}

}  // namespace

extern "C" {

srtc_status srtc_features(srtc_ctx *ctx, srtc_semiring sr, const srtc_tensor *A, const srtc_tensor *B, float *out,
                          void *stream) {
  return guard(ctx, [&] {
    if (!out) fail(SRTC_ERR_ARG, "features: null output");
    const CsrView a = matrix_view(A, "A"), b = matrix_view(B, "B");
    if (A->dtype != B->dtype) fail(SRTC_ERR_DTYPE, "A and B value types differ");
    ctx->c.stream = (hipStream_t)stream;
    spgemm_features(&ctx->c, sr, A->dtype, a, b, out, (hipStream_t)stream);
  });
}

srtc_status srtc_autotune(srtc_ctx *ctx, srtc_semiring sr, const void *add_id, const srtc_tensor *A,
                          const srtc_tensor *B, int32_t reps, srtc_schedule *best, float *times_ms, void *stream) {
  return guard(ctx, [&] {
    const CsrView a = matrix_view(A, "A"), b = matrix_view(B, "B");
    if (A->dtype != B->dtype) fail(SRTC_ERR_DTYPE, "A and B value types differ");
    const int dt = A->dtype;
    const IdVal id = make_id_public(sr, dt, add_id);
    if (reps < 1) reps = 1;
    Ctx *c = &ctx->c;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    hipEvent_t e0, e1;
    SRTC_HIP(hipEventCreate(&e0));
    SRTC_HIP(hipEventCreate(&e1));
    std::vector<float> med(SRTC_NUM_SCHEDULES, 0.f);
    for (int k = 0; k < SRTC_NUM_SCHEDULES; k++) {
      std::vector<float> ts;
      for (int r = 0; r <= reps; r++) {
        CsrOut out;
        SRTC_HIP(hipEventRecord(e0, s));
        spgemm(c, sr, dt, id, a, b, k, 1, &out, nullptr, s);
        SRTC_HIP(hipEventRecord(e1, s));
        SRTC_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SRTC_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (r > 0) ts.push_back(ms);  // the first run is the warm-up
      }
      std::sort(ts.begin(), ts.end());
      const size_t h = ts.size() / 2;
      med[k] = ts.size() % 2 ? ts[h] : 0.5f * (ts[h - 1] + ts[h]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int arg = 0;
    for (int k = 1; k < SRTC_NUM_SCHEDULES; k++)
      if (med[k] < med[arg]) arg = k;
    float feat[SRTC_NUM_FEATURES];
    spgemm_features(c, sr, dt, a, b, feat, s);
    c->tune_cache[tune_key(sr, dt, feat)] = arg;
    if (best) *best = arg;
    if (times_ms)
      for (int k = 0; k < SRTC_NUM_SCHEDULES; k++) times_ms[k] = med[k];
  });
}

}  // extern "C"
