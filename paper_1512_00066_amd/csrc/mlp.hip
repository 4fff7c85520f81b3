// Learned schedule selector: a 32 -> 64 -> 64 -> K multilayer perceptron
// (ReLU) trained with the mean-squared error on per-schedule log2 times and
// Adam, with forward, backward and update as HIP kernels.
//
// The paper selects among algorithms with performance models scaled by the
// nonzero fraction and a tunable prefactor, and names automatically
// adjusted performance models as future work (Sections 5.1 and 7); this
// network is such a model, fitted to timings the library itself measures.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "internal.hpp"

namespace srtc {

namespace {
constexpr int IN = SRTC_NUM_FEATURES, H = 64, K = SRTC_NUM_SCHEDULES;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * IN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + K * H, NPARAM = OFF_B3 + K;
}  // namespace

struct Mlp {
  std::vector<float> params, m1, m2;  // host copies (weights, Adam moments)
  float mean[IN], stdv[IN];
  int64_t step = 0;
  // device copy for selection: params, then mean and stdv (uploaded once per
  // training or load; the network is small, so it lives outside the
  // allocator callback and is freed with the network)
  float *dev = nullptr;
  int dev_id = -1;
};

void mlp_destroy(Mlp *m) {
  if (!m) return;
  if (m->dev) (void)hipFree(m->dev);
  delete m;
}

namespace {

// One 64-thread block per sample: activations, output, and (with targets)
// the per-sample deltas.
__global__ void __launch_bounds__(64) mlp_sample(const float *__restrict__ P, const float *__restrict__ X,
                                                 const float *__restrict__ T, int n, float *__restrict__ Y,
                                                 float *__restrict__ H1, float *__restrict__ H2,
                                                 float *__restrict__ DZ1, float *__restrict__ DZ2,
                                                 float *__restrict__ DY, float *__restrict__ lsum) {
  __shared__ float x[IN], h1[H], h2[H], dy[K], dz2[H];
  const int s = blockIdx.x, t = threadIdx.x;
  if (s >= n) return;
  if (t < IN) x[t] = X[(int64_t)s * IN + t];
  __syncthreads();
  float z1 = P[OFF_B1 + t];
  for (int i = 0; i < IN; i++) z1 += P[OFF_W1 + t * IN + i] * x[i];
  h1[t] = z1 > 0.f ? z1 : 0.f;
  __syncthreads();
  float z2 = P[OFF_B2 + t];
  for (int i = 0; i < H; i++) z2 += P[OFF_W2 + t * H + i] * h1[i];
  h2[t] = z2 > 0.f ? z2 : 0.f;
  __syncthreads();
  float y = 0.f;
  if (t < K) {
    y = P[OFF_B3 + t];
    for (int i = 0; i < H; i++) y += P[OFF_W3 + t * H + i] * h2[i];
    Y[(int64_t)s * K + t] = y;
  }
  if (!T) return;
  float e = 0.f;
  if (t < K) {
    const float d = y - T[(int64_t)s * K + t];
    e = d * d;
    dy[t] = 2.f * d / (float)(n * K);
    DY[(int64_t)s * K + t] = dy[t];
  }
  e = wave_sum(e);
  if (t == 0) lsum[s] = e;
  __syncthreads();
  float g2 = 0.f;
  for (int k = 0; k < K; k++) g2 += P[OFF_W3 + k * H + t] * dy[k];
  g2 = z2 > 0.f ? g2 : 0.f;
  dz2[t] = g2;
  DZ2[(int64_t)s * H + t] = g2;
  H1[(int64_t)s * H + t] = h1[t];
  H2[(int64_t)s * H + t] = h2[t];
  __syncthreads();
  float g1 = 0.f;
  for (int o = 0; o < H; o++) g1 += P[OFF_W2 + o * H + t] * dz2[o];
  g1 = z1 > 0.f ? g1 : 0.f;
  DZ1[(int64_t)s * H + t] = g1;
}

// One thread per parameter: sum of per-sample contributions in sample order.
__global__ void mlp_grads(const float *__restrict__ X, const float *__restrict__ H1, const float *__restrict__ H2,
                          const float *__restrict__ DZ1, const float *__restrict__ DZ2, const float *__restrict__ DY,
                          int n, float *__restrict__ G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  float acc = 0.f;
  if (p < OFF_B1) {
    const int o = (p - OFF_W1) / IN, i = (p - OFF_W1) % IN;
    for (int s = 0; s < n; s++) acc += DZ1[(int64_t)s * H + o] * X[(int64_t)s * IN + i];
  } else if (p < OFF_W2) {
    const int o = p - OFF_B1;
    for (int s = 0; s < n; s++) acc += DZ1[(int64_t)s * H + o];
  } else if (p < OFF_B2) {
    const int o = (p - OFF_W2) / H, i = (p - OFF_W2) % H;
    for (int s = 0; s < n; s++) acc += DZ2[(int64_t)s * H + o] * H1[(int64_t)s * H + i];
  } else if (p < OFF_W3) {
    const int o = p - OFF_B2;
    for (int s = 0; s < n; s++) acc += DZ2[(int64_t)s * H + o];
  } else if (p < OFF_B3) {
    const int o = (p - OFF_W3) / H, i = (p - OFF_W3) % H;
    for (int s = 0; s < n; s++) acc += DY[(int64_t)s * K + o] * H2[(int64_t)s * H + i];
  } else {
    const int o = p - OFF_B3;
    for (int s = 0; s < n; s++) acc += DY[(int64_t)s * K + o];
  }
  G[p] = acc;
}

__global__ void mlp_loss_reduce(const float *__restrict__ lsum, int n, float *__restrict__ loss) {
  float a = 0.f;
  for (int s = threadIdx.x; s < n; s += 64) a += lsum[s];
  a = wave_sum(a);
  if (threadIdx.x == 0) *loss = a / (float)(n * K);
}

__global__ void gather_rows(const float *__restrict__ src, const int32_t *__restrict__ idx, int n, int width,
                            float *__restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * width) return;
  const int64_t r = t / width, q = t % width;
  dst[t] = src[(int64_t)idx[r] * width + q];
}

// Adam (Kingma and Ba): first and second moment estimates, bias corrections
// c1 = 1 - b1^t and c2 = 1 - b2^t for step t, then the scaled step.
__global__ void adam_update(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ M1,
                            float *__restrict__ M2, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float g = G[p];
  const float m = b1 * M1[p] + (1.f - b1) * g;
  const float v = b2 * M2[p] + (1.f - b2) * g * g;
  M1[p] = m;
  M2[p] = v;
  P[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Selection: one 64-thread block standardizes the features with the
// network's statistics, evaluates the network and writes the arg-min of the
// predicted (centred log2) times.
__global__ void __launch_bounds__(64) mlp_select_kernel(const float *__restrict__ P, const float *__restrict__ mean,
                                                        const float *__restrict__ stdv, const float *__restrict__ feat,
                                                        int32_t *__restrict__ pick) {
  __shared__ float x[IN], h1[H], h2[H], y[K];
  const int t = threadIdx.x;
  if (t < IN) x[t] = (feat[t] - mean[t]) / stdv[t];
  __syncthreads();
  float z1 = P[OFF_B1 + t];
  for (int i = 0; i < IN; i++) z1 += P[OFF_W1 + t * IN + i] * x[i];
  h1[t] = z1 > 0.f ? z1 : 0.f;
  __syncthreads();
  float z2 = P[OFF_B2 + t];
  for (int i = 0; i < H; i++) z2 += P[OFF_W2 + t * H + i] * h1[i];
  h2[t] = z2 > 0.f ? z2 : 0.f;
  __syncthreads();
  if (t < K) {
    float v = P[OFF_B3 + t];
    for (int i = 0; i < H; i++) v += P[OFF_W3 + t * H + i] * h2[i];
    y[t] = v;
  }
  __syncthreads();
  if (t == 0) {
    int best = 0;
    for (int k = 1; k < K; k++)
      if (y[k] < y[best]) best = k;
    *pick = best;
  }
}

// Upload the network (parameters and feature statistics) for selection.
void mlp_to_device(Ctx *c, Mlp *m) {
  const size_t bytes = 4ull * (NPARAM + 2 * IN);
  if (!m->dev || m->dev_id != c->device) {
    if (m->dev) (void)hipFree(m->dev);
    m->dev = nullptr;
    if (hipMalloc(&m->dev, bytes) != hipSuccess) {
      m->dev = nullptr;
      fail(SRTC_ERR_OOM, "selector network: device allocation failed");
    }
    m->dev_id = c->device;
  }
  std::vector<float> h(NPARAM + 2 * IN);
  std::copy(m->params.begin(), m->params.end(), h.begin());
  std::copy(m->mean, m->mean + IN, h.begin() + NPARAM);
  std::copy(m->stdv, m->stdv + IN, h.begin() + NPARAM + IN);
  SRTC_HIP(hipMemcpy(m->dev, h.data(), bytes, hipMemcpyHostToDevice));
}

struct Scratch {
  Buf X, T, Y, H1, H2, DZ1, DZ2, DY, L, G;
  Scratch(Ctx *c, int n)
      : X(c, 4ull * n * IN), T(c, 4ull * n * K), Y(c, 4ull * n * K), H1(c, 4ull * n * H), H2(c, 4ull * n * H),
        DZ1(c, 4ull * n * H), DZ2(c, 4ull * n * H), DY(c, 4ull * n * K), L(c, 4ull * std::max(n, 1) + 256),
        G(c, 4ull * NPARAM) {}
};

void forward_dev(const float *P, const float *X, int n, float *Y, hipStream_t s) {
  if (n <= 0) return;
  mlp_sample<<<n, 64, 0, s>>>(P, X, nullptr, n, Y, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  SRTC_LAUNCH_CHECK("mlp_sample");
}

void loss_grad_dev(const float *P, const float *X, const float *T, int n, float *Y, float *H1, float *H2, float *DZ1,
                   float *DZ2, float *DY, float *lsum, float *loss, float *G, hipStream_t s) {
  mlp_sample<<<n, 64, 0, s>>>(P, X, T, n, Y, H1, H2, DZ1, DZ2, DY, lsum);
  SRTC_LAUNCH_CHECK("mlp_sample");
  mlp_grads<<<(NPARAM + 255) / 256, 256, 0, s>>>(X, H1, H2, DZ1, DZ2, DY, n, G);
  SRTC_LAUNCH_CHECK("mlp_grads");
  mlp_loss_reduce<<<1, 64, 0, s>>>(lsum, n, loss);
  SRTC_LAUNCH_CHECK("mlp_loss_reduce");
}

uint64_t splitmix(uint64_t &state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double unif(uint64_t &st) { return (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0); }

void normalize(const Mlp *m, const float *in, float *out, int n) {
  for (int s = 0; s < n; s++)
    for (int i = 0; i < IN; i++) out[(int64_t)s * IN + i] = (in[(int64_t)s * IN + i] - m->mean[i]) / m->stdv[i];
}

}  // namespace
}  // namespace srtc

using namespace srtc;

extern "C" {

srtc_status srtc_mlp_forward(srtc_ctx *ctx, const float *params, const float *X, int32_t n, float *Y, void *stream) {
  return guard(ctx, [&] {
    if (!params || !X || !Y || n < 0) fail(SRTC_ERR_ARG, "mlp_forward: bad arguments");
    ctx->c.stream = (hipStream_t)stream;
    forward_dev(params, X, n, Y, (hipStream_t)stream);
  });
}

srtc_status srtc_mlp_loss_grad(srtc_ctx *ctx, const float *params, const float *X, const float *T, int32_t n,
                               float *loss, float *grads, void *stream) {
  return guard(ctx, [&] {
    if (!params || !X || !T || !loss || !grads || n <= 0) fail(SRTC_ERR_ARG, "mlp_loss_grad: bad arguments");
    Ctx *c = &ctx->c;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    Scratch w(c, n);
    loss_grad_dev(params, X, T, n, w.Y.as<float>(), w.H1.as<float>(), w.H2.as<float>(), w.DZ1.as<float>(),
                  w.DZ2.as<float>(), w.DY.as<float>(), w.L.as<float>(), loss, grads, s);
  });
}

srtc_status srtc_selector_train(srtc_ctx *ctx, const float *X, const float *T, int32_t nsamples,
                                const srtc_train_cfg *cfg, float *final_loss, void *stream) {
  return guard(ctx, [&] {
    if (!X || !T || nsamples <= 0 || !cfg) fail(SRTC_ERR_ARG, "selector_train: bad arguments");
    if (cfg->batch <= 0 || cfg->batch > 1024 || cfg->epochs < 0) fail(SRTC_ERR_ARG, "selector_train: batch 1..1024");
    Ctx *c = &ctx->c;
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    Mlp *m = c->mlp;
    uint64_t rng = cfg->seed ^ 0x5EEDull;
    if (!m) {
      m = new Mlp();
      m->params.assign(NPARAM, 0.f);
      m->m1.assign(NPARAM, 0.f);
      m->m2.assign(NPARAM, 0.f);
      // He-uniform initialization, zero biases
      auto init = [&](int off, int fan_in, int count) {
        const double a = std::sqrt(6.0 / fan_in);
        for (int q = 0; q < count; q++) m->params[off + q] = (float)((2.0 * unif(rng) - 1.0) * a);
      };
      init(OFF_W1, IN, H * IN);
      init(OFF_W2, H, H * H);
      init(OFF_W3, H, K * H);
      // feature standardization from the training set
      for (int i = 0; i < IN; i++) {
        double mu = 0, sq = 0;
        for (int t = 0; t < nsamples; t++) mu += X[(int64_t)t * IN + i];
        mu /= nsamples;
        for (int t = 0; t < nsamples; t++) {
          const double d = X[(int64_t)t * IN + i] - mu;
          sq += d * d;
        }
        m->mean[i] = (float)mu;
        m->stdv[i] = (float)std::max(1e-6, std::sqrt(sq / nsamples));
      }
      c->mlp = m;
    }
    std::vector<float> Xn((size_t)nsamples * IN);
    normalize(m, X, Xn.data(), nsamples);
    const int bsz = cfg->batch;
    Buf P(c, 4ull * NPARAM), M1(c, 4ull * NPARAM), M2(c, 4ull * NPARAM), loss(c, 256);
    Scratch w(c, bsz);
    SRTC_HIP(hipMemcpyAsync(P.p, m->params.data(), 4ull * NPARAM, hipMemcpyHostToDevice, s));
    SRTC_HIP(hipMemcpyAsync(M1.p, m->m1.data(), 4ull * NPARAM, hipMemcpyHostToDevice, s));
    SRTC_HIP(hipMemcpyAsync(M2.p, m->m2.data(), 4ull * NPARAM, hipMemcpyHostToDevice, s));
    Buf Xd(c, 4ull * nsamples * IN), Td(c, 4ull * nsamples * K);
    SRTC_HIP(hipMemcpyAsync(Xd.p, Xn.data(), 4ull * nsamples * IN, hipMemcpyHostToDevice, s));
    SRTC_HIP(hipMemcpyAsync(Td.p, T, 4ull * nsamples * K, hipMemcpyHostToDevice, s));
    std::vector<int> order(nsamples);
    for (int t = 0; t < nsamples; t++) order[t] = t;
    float last = 0.f;
    Buf ord(c, 4ull * nsamples);
    for (int ep = 0; ep < cfg->epochs; ep++) {
      for (int t = nsamples - 1; t > 0; t--) std::swap(order[t], order[splitmix(rng) % (uint64_t)(t + 1)]);
      {
        void *pin = c->host_scratch(4ull * nsamples);
        memcpy(pin, order.data(), 4ull * nsamples);
        SRTC_HIP(hipMemcpyAsync(ord.p, pin, 4ull * nsamples, hipMemcpyHostToDevice, s));
        SRTC_HIP(hipStreamSynchronize(s));
      }
      double tot = 0;
      int nb = 0;
      for (int b0 = 0; b0 < nsamples; b0 += bsz) {
        const int nbt = std::min(bsz, nsamples - b0);
        gather_rows<<<(nbt * IN + 255) / 256, 256, 0, s>>>(Xd.as<float>(), ord.as<int32_t>() + b0, nbt, IN, w.X.as<float>());
        gather_rows<<<(nbt * K + 255) / 256, 256, 0, s>>>(Td.as<float>(), ord.as<int32_t>() + b0, nbt, K, w.T.as<float>());
        SRTC_LAUNCH_CHECK("gather_rows");
        loss_grad_dev(P.as<float>(), w.X.as<float>(), w.T.as<float>(), nbt, w.Y.as<float>(), w.H1.as<float>(),
                      w.H2.as<float>(), w.DZ1.as<float>(), w.DZ2.as<float>(), w.DY.as<float>(), w.L.as<float>(),
                      loss.as<float>() + (nb % 32), w.G.as<float>(), s);
        m->step++;
        const float c1 = 1.f - (float)std::pow((double)cfg->beta1, (double)m->step);
        const float c2 = 1.f - (float)std::pow((double)cfg->beta2, (double)m->step);
        adam_update<<<(NPARAM + 255) / 256, 256, 0, s>>>(P.as<float>(), w.G.as<float>(), M1.as<float>(), M2.as<float>(),
                                                         cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, c1, c2);
        SRTC_LAUNCH_CHECK("adam_update");
        nb++;
        if (nb % 32 == 0 || b0 + bsz >= nsamples) {
          float hl[32];
          const int cnt = nb % 32 == 0 ? 32 : nb % 32;
          read_to_host(c, hl, loss.p, 4ull * cnt, s);
          for (int q = 0; q < cnt; q++) tot += hl[q];
        }
      }
      last = (float)(tot / std::max(nb, 1));
    }
    read_to_host(c, m->params.data(), P.p, 4ull * NPARAM, s);
    read_to_host(c, m->m1.data(), M1.p, 4ull * NPARAM, s);
    read_to_host(c, m->m2.data(), M2.p, 4ull * NPARAM, s);
    mlp_to_device(c, m);
    if (final_loss) *final_loss = last;
  });
}

srtc_status srtc_select(srtc_ctx *ctx, const float *features, srtc_schedule *schedule_out) {
  return guard(ctx, [&] {
    if (!features || !schedule_out) fail(SRTC_ERR_ARG, "select: null");
    Ctx *c = &ctx->c;
    Mlp *m = c->mlp;
    if (!m) fail(SRTC_ERR_UNSUPPORTED, "no selector network loaded");
    if (!m->dev || m->dev_id != c->device) mlp_to_device(c, m);
    hipStream_t s = c->stream;  // the caller's stream when nested in a contraction
    // features in, pick out: one 32-float upload, one kernel, one int read
    Buf io(c, 4ull * IN + 64);
    float *pin = (float *)c->host_scratch(4ull * IN);
    memcpy(pin, features, 4ull * IN);
    SRTC_HIP(hipMemcpyAsync(io.p, pin, 4ull * IN, hipMemcpyHostToDevice, s));
    int32_t *pick = reinterpret_cast<int32_t *>(io.as<char>() + 4ull * IN);
    mlp_select_kernel<<<1, 64, 0, s>>>(m->dev, m->dev + NPARAM, m->dev + NPARAM + IN, io.as<float>(), pick);
    SRTC_LAUNCH_CHECK("mlp_select_kernel");
    int32_t best = 0;
    read_to_host(c, &best, pick, sizeof(best), s);
    *schedule_out = best;
  });
}

srtc_status srtc_mlp_adam_step(srtc_ctx *ctx, float *params, const float *grads, float *m1, float *m2, int64_t step,
                               float lr, float beta1, float beta2, float eps, void *stream) {
  return guard(ctx, [&] {
    if (!params || !grads || !m1 || !m2 || step < 1) fail(SRTC_ERR_ARG, "mlp_adam_step: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    ctx->c.stream = s;
    // the same bias corrections as the training loop
    const float c1 = 1.f - (float)std::pow((double)beta1, (double)step);
    const float c2 = 1.f - (float)std::pow((double)beta2, (double)step);
    adam_update<<<(NPARAM + 255) / 256, 256, 0, s>>>(params, grads, m1, m2, lr, beta1, beta2, eps, c1, c2);
    SRTC_LAUNCH_CHECK("adam_update");
  });
}

srtc_status srtc_selector_save(srtc_ctx *ctx, const char *path) {
  return guard(ctx, [&] {
    Ctx *c = &ctx->c;
    if (!path) fail(SRTC_ERR_ARG, "null path");
    if (!c->mlp) fail(SRTC_ERR_UNSUPPORTED, "no selector network");
    FILE *f = fopen(path, "wb");
    if (!f) fail(SRTC_ERR_ARG, "cannot open file");
    const uint32_t hdr[4] = {0x53525443u, 1u, (uint32_t)K, (uint32_t)NPARAM};
    bool ok = fwrite(hdr, sizeof(hdr), 1, f) == 1;
    ok = ok && fwrite(c->mlp->params.data(), 4, NPARAM, f) == (size_t)NPARAM;
    ok = ok && fwrite(c->mlp->mean, 4, IN, f) == (size_t)IN && fwrite(c->mlp->stdv, 4, IN, f) == (size_t)IN;
    ok = ok && fwrite(c->mlp->m1.data(), 4, NPARAM, f) == (size_t)NPARAM;
    ok = ok && fwrite(c->mlp->m2.data(), 4, NPARAM, f) == (size_t)NPARAM;
    ok = ok && fwrite(&c->mlp->step, 8, 1, f) == 1;
    fclose(f);
    if (!ok) fail(SRTC_ERR_ARG, "write failed");
  });
}

srtc_status srtc_selector_load(srtc_ctx *ctx, const char *path) {
  return guard(ctx, [&] {
    Ctx *c = &ctx->c;
    if (!path) fail(SRTC_ERR_ARG, "null path");
    FILE *f = fopen(path, "rb");
    if (!f) fail(SRTC_ERR_ARG, "cannot open file");
    uint32_t hdr[4];
    Mlp *m = new Mlp();
    m->params.assign(NPARAM, 0.f);
    m->m1.assign(NPARAM, 0.f);
    m->m2.assign(NPARAM, 0.f);
    bool ok = fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == 0x53525443u && hdr[2] == (uint32_t)K &&
              hdr[3] == (uint32_t)NPARAM;
    ok = ok && fread(m->params.data(), 4, NPARAM, f) == (size_t)NPARAM;
    ok = ok && fread(m->mean, 4, IN, f) == (size_t)IN && fread(m->stdv, 4, IN, f) == (size_t)IN;
    ok = ok && fread(m->m1.data(), 4, NPARAM, f) == (size_t)NPARAM;
    ok = ok && fread(m->m2.data(), 4, NPARAM, f) == (size_t)NPARAM;
    ok = ok && fread(&m->step, 8, 1, f) == 1;
    fclose(f);
    if (!ok) {
      delete m;
      fail(SRTC_ERR_FORMAT, "not a selector file");
    }
    mlp_destroy(c->mlp);
    c->mlp = m;
    mlp_to_device(c, m);
  });
}

}  // extern "C"
