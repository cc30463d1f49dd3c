// Learned cost model: features, training on device timings, persistence.
//
// The paper's shortest path is weighted by a measured tuning profile of
// section times (section 2, third paragraph).  Measuring every (section,
// candidate layout) pair is what planning time is spent on; the learned
// model predicts ln(time) of a section under a layout from 16 features and
// the planner uses its predictions as the edge weights instead.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "adha_impl.h"

namespace adha {

double analytic_bytes_per_record(const SectionDesc &s, const LayoutDesc &l);
double analytic_section_us(const SectionDesc &s, const LayoutDesc &l);
adha_status fill_uniform_index(int32_t *idx, uint64_t count, int64_t n, uint64_t seed, hipStream_t stream);
std::vector<std::vector<int>> ods_parts(const std::vector<SectionDesc> &secs, size_t first, size_t last,
                                        const Shape &sh, uint32_t cap);

// Wide loads per neighbour when a gather's reads all sit in one interleaved
// group and span at most 64 bytes (the span-gather kernel); 0 otherwise.
static uint32_t span_loads(const SectionDesc &s, const LayoutDesc &l) {
  if (s.degree == 0 || s.rd.empty()) return 0;
  const uint32_t g = l.group_of[s.rd[0]];
  for (int f : s.rd)
    if (l.group_of[f] != g) return 0;
  const Group &G = l.groups[g];
  if (G.T != 1) return 0;
  uint32_t lo = ~0u, hi = 0;
  for (int f : s.rd) {
    lo = std::min(lo, l.p[f]);
    hi = std::max(hi, l.p[f] + l.shape.ebytes[f]);
  }
  const uint32_t A = G.S % 16 == 0 ? 16 : G.S % 8 == 0 ? 8 : 4;
  const uint32_t lo_a = lo / A * A, nvec = (hi - lo_a + A - 1) / A;
  return nvec * A / 4 > 16 ? 0 : nvec;
}

// Features (all scaled to roughly [0, 1]).  They describe the section and
// the groups it touches, not the layout as a whole: groups the section does
// not touch do not change its time.
//  0 log2 N / 24            1 |R| / 16               2 |W| / 2
//  3 d / 32                 4 log2(1 + read bytes) / 8   5 log2(1 + write bytes) / 8
//  6 groups holding R / 16  7 groups holding W / 2
//  8 span gather applies    9 span loads per neighbour / 16
//  10 share of R in one-field groups
//  11 share of R in interleaved groups of several fields
//  12 share of R in tiled groups of several fields
//  13 share of W in groups of several fields
//  14 gathers: log2(N * record bytes of the groups holding R) / 32, the
//     footprint the random reads range over (it decides which cache level
//     holds them); direct sections: 0
//  15 log2(analytic bytes per record) / 12
void section_features(const SectionDesc &s, const LayoutDesc &l, float *out) {
  double rb = 0, wb = 0, r_one = 0, r_inter = 0, r_tiled = 0, w_multi = 0;
  for (int f : s.rd) {
    rb += l.shape.ebytes[f];
    const Group &G = l.groups[l.group_of[f]];
    if (G.fields.size() == 1)
      r_one += 1;
    else if (G.T == 1)
      r_inter += 1;
    else
      r_tiled += 1;
  }
  for (int f : s.wr) {
    wb += l.shape.ebytes[f];
    if (l.groups[l.group_of[f]].fields.size() > 1) w_multi += 1;
  }
  std::vector<char> rg(l.groups.size(), 0), wg(l.groups.size(), 0);
  for (int f : s.rd) rg[l.group_of[f]] = 1;
  for (int f : s.wr) wg[l.group_of[f]] = 1;
  double nrg = 0, nwg = 0, foot = 0;
  for (size_t g = 0; g < l.groups.size(); ++g) {
    nrg += rg[g];
    nwg += wg[g];
    if (rg[g]) foot += (double)l.groups[g].S;
  }
  foot *= (double)l.shape.n;
  const double nr = (double)std::max<size_t>(1, s.rd.size()), nw = (double)std::max<size_t>(1, s.wr.size());
  const uint32_t sl = span_loads(s, l);
  const double v[ADHA_N_FEATURES] = {
      std::log2((double)std::max<int64_t>(1, l.shape.n)) / 24.0,
      s.rd.size() / 16.0,
      s.wr.size() / 2.0,
      s.degree / 32.0,
      std::log2(1.0 + rb) / 8.0,
      std::log2(1.0 + wb) / 8.0,
      nrg / 16.0,
      nwg / 2.0,
      sl ? 1.0 : 0.0,
      sl / 16.0,
      r_one / nr,
      r_inter / nr,
      r_tiled / nr,
      w_multi / nw,
      s.degree ? std::log2(std::max(1.0, foot)) / 32.0 : 0.0,
      std::log2(std::max(1.0, analytic_bytes_per_record(s, l))) / 12.0};
  for (int i = 0; i < ADHA_N_FEATURES; ++i) out[i] = (float)v[i];
}

// The network predicts the log of the ratio between a section's time and
// the analytic model's estimate; base_us holds those estimates.
adha_status predict_costs(Ctx *ctx, const std::vector<std::vector<float>> &feats, const std::vector<double> &base_us,
                          std::vector<double> *us, hipStream_t stream) {
  if (!ctx->has_model) return fail(ADHA_ERR_STATE, "no cost model loaded");
  const uint32_t B = (uint32_t)feats.size();
  us->assign(B, 0.0);
  if (B == 0) return ADHA_OK;
  std::vector<float> x((size_t)B * ADHA_N_FEATURES), y(B);
  for (uint32_t i = 0; i < B; ++i) memcpy(&x[(size_t)i * ADHA_N_FEATURES], feats[i].data(), ADHA_N_FEATURES * 4);
  // the context keeps the parameters on the device (uploaded once per
  // model) and grow-only input and output buffers
  const uint32_t K = ctx->n_models;
  if (!ctx->mlp_params) ADHA_HIP(hipMalloc((void **)&ctx->mlp_params, (size_t)kMaxEnsemble * ADHA_MLP_PARAMS * 4));
  if (!ctx->mlp_params_ok) {
    ADHA_HIP(hipMemcpy(ctx->mlp_params, ctx->model.data(), (size_t)K * ADHA_MLP_PARAMS * 4, hipMemcpyHostToDevice));
    ctx->mlp_params_ok = true;
  }
  if (ctx->mlp_io_cap < B) {
    ADHA_HIP(hipStreamSynchronize(stream));
    if (ctx->mlp_x) (void)hipFree(ctx->mlp_x);
    if (ctx->mlp_y) (void)hipFree(ctx->mlp_y);
    ctx->mlp_x = ctx->mlp_y = nullptr;
    ctx->mlp_io_cap = 0;
    const uint32_t cap = std::max<uint32_t>(B, 1024);
    ADHA_HIP(hipMalloc((void **)&ctx->mlp_x, (size_t)cap * ADHA_N_FEATURES * 4));
    ADHA_HIP(hipMalloc((void **)&ctx->mlp_y, (size_t)kMaxEnsemble * cap * 4));
    ctx->mlp_io_cap = cap;
  }
  ADHA_HIP(hipMemcpyAsync(ctx->mlp_x, x.data(), x.size() * 4, hipMemcpyHostToDevice, stream));
  for (uint32_t k = 0; k < K; ++k)
    ADHA_TRY(mlp_forward(ctx, ctx->mlp_params + (size_t)k * ADHA_MLP_PARAMS, ctx->mlp_x, B,
                         ctx->mlp_y + (size_t)k * ctx->mlp_io_cap, stream));
  std::vector<float> yk((size_t)K * ctx->mlp_io_cap);
  ADHA_HIP(hipMemcpyAsync(yk.data(), ctx->mlp_y, yk.size() * 4, hipMemcpyDeviceToHost, stream));
  ADHA_HIP(hipStreamSynchronize(stream));
  // the networks' mean prediction of the log ratio
  for (uint32_t i = 0; i < B; ++i) {
    double m = 0.0;
    for (uint32_t k = 0; k < K; ++k) m += yk[(size_t)k * ctx->mlp_io_cap + i];
    y[i] = (float)(m / K);
  }
  for (uint32_t i = 0; i < B; ++i) (*us)[i] = base_us[i] * std::exp((double)y[i]);
  return ADHA_OK;
}

// SplitMix64 (Steele, Lea, Flood 2014), used to draw training sections.
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  uint32_t below(uint32_t n) { return (uint32_t)(((next() >> 32) * n) >> 32); }
  double unit() { return (next() >> 11) * 0x1.0p-53; }
};

static Shape training_shape(int64_t n) {
  Shape sh;
  sh.n = n;
  for (int f = 0; f < 32; ++f) {
    sh.dtype.push_back(f < 20 ? ADHA_F32 : f < 28 ? ADHA_I32 : ADHA_F64);
    sh.ebytes.push_back(f < 28 ? 4 : 8);
  }
  return sh;
}

static SectionDesc random_section(Rng &g, const Shape &sh) {
  SectionDesc d;
  d.shape = sh;
  d.op = ADHA_OP_GEN;
  const int F = sh.nfields();
  std::vector<int> perm(F);
  for (int f = 0; f < F; ++f) perm[f] = f;
  for (int k = F - 1; k > 0; --k) std::swap(perm[k], perm[g.below(k + 1)]);
  const uint32_t nr = 1 + g.below(16), nw = 1 + g.below(2);
  d.rd.assign(perm.begin(), perm.begin() + nr);
  d.wr.assign(perm.begin() + nr, perm.begin() + nr + nw);
  std::sort(d.rd.begin(), d.rd.end());
  std::sort(d.wr.begin(), d.wr.end());
  d.degree = g.below(2) ? 0 : 1 + g.below(32);
  return d;
}

static LayoutDesc random_layout(Rng &g, const Shape &sh, const SectionDesc &sec) {
  switch (g.below(8)) {
    case 0: return layout_aos(sh);
    case 1: return layout_soa(sh);
    case 2: return layout_aos(sh, 64);
    case 3: {
      static const uint32_t caps[] = {16, 32, 64, 128};
      auto parts = ods_parts({sec}, 0, 0, sh, caps[g.below(4)]);
      return layout_from_parts(sh, parts, g.below(2) ? 64 : 1);
    }
    case 4:
    case 5: {
      // the kind of layout the planner's catalogue holds: the ODS of a run of
      // sections that includes this one
      std::vector<SectionDesc> run;
      const uint32_t others = 1 + g.below(3), at = g.below(others + 1);
      for (uint32_t q = 0; q <= others; ++q) run.push_back(q == at ? sec : random_section(g, sh));
      auto parts = ods_parts(run, 0, run.size() - 1, sh, 64);
      return layout_from_parts(sh, parts, g.below(2) ? 64 : 1);
    }
    default: {
      // a random partition into consecutive chunks of 2..8 fields
      std::vector<std::vector<int>> parts;
      const int F = sh.nfields();
      for (int f = 0; f < F;) {
        int c = 2 + (int)g.below(7);
        std::vector<int> p;
        for (int q = f; q < std::min(F, f + c); ++q) p.push_back(q);
        if (p.size() > 1) parts.push_back(p);
        f += c;
      }
      return layout_from_parts(sh, parts, g.below(2) ? 64 : 1);
    }
  }
}

static uint64_t fnv1a(const void *p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  const uint8_t *b = (const uint8_t *)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

}  // namespace adha

using namespace adha;

extern "C" {

adha_status adha_features(const adha_section *sec, const adha_layout *l, float *out16) {
  if (!sec || !l || !out16) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!sec->d.shape.same(l->d.shape)) return fail(ADHA_ERR_INVALID, "section and layout describe different structs");
  section_features(sec->d, l->d, out16);
  return ADHA_OK;
}

adha_status adha_section_effective_bytes(const adha_section *sec, const adha_layout *l, double *out) {
  if (!sec || !l || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!sec->d.shape.same(l->d.shape)) return fail(ADHA_ERR_INVALID, "section and layout describe different structs");
  *out = (double)l->d.shape.n * analytic_bytes_per_record(sec->d, l->d);
  return ADHA_OK;
}

static bool dev_ok(const void *p) { return p && ((uintptr_t)p & 3u) == 0; }

adha_status adha_mlp_forward(adha_ctx *ctx, const float *params, const float *x, uint32_t batch, float *y,
                             void *stream) {
  if (!ctx || !dev_ok(params) || !dev_ok(x) || !dev_ok(y)) return fail(ADHA_ERR_INVALID, "NULL or misaligned argument");
  DeviceGuard g(ctx->c.device);
  return mlp_forward(&ctx->c, params, x, batch, y, (hipStream_t)stream);
}

adha_status adha_mlp_backward(adha_ctx *ctx, const float *params, const float *x, const float *target,
                              uint32_t batch, float *grad, float *loss, void *stream) {
  if (!ctx || !dev_ok(params) || !dev_ok(x) || !dev_ok(target) || !dev_ok(grad))
    return fail(ADHA_ERR_INVALID, "NULL or misaligned argument");
  if (batch == 0 || batch > (1u << 20)) return fail(ADHA_ERR_INVALID, "batch %u not in [1, 2^20]", batch);
  DeviceGuard g(ctx->c.device);
  hipStream_t st = (hipStream_t)stream;
  float *s = nullptr;
  ADHA_HIP(hipMallocAsync((void **)&s, mlp_scratch_floats(batch) * 4, st));
  adha_status r = mlp_backward(&ctx->c, params, x, target, batch, grad, loss, s, mlp_scratch_floats(batch), st);
  (void)hipFreeAsync(s, st);
  return r;
}

adha_status adha_mlp_adam(adha_ctx *ctx, float *params, const float *grad, float *m, float *v, float lr, float b1,
                          float b2, float eps, uint32_t t, void *stream) {
  if (!ctx || !dev_ok(params) || !dev_ok(grad) || !dev_ok(m) || !dev_ok(v))
    return fail(ADHA_ERR_INVALID, "NULL or misaligned argument");
  DeviceGuard g(ctx->c.device);
  return mlp_adam(&ctx->c, params, grad, m, v, lr, b1, b2, eps, t, (hipStream_t)stream);
}

adha_status adha_train_opts_default(adha_train_opts *o) {
  if (!o) return fail(ADHA_ERR_INVALID, "NULL argument");
  o->n_samples = 2000;
  o->epochs = 300;
  o->batch = 256;
  o->lr = 1e-3f;
  o->seed = 5;
  o->min_log2_n = 16;
  o->max_log2_n = 22;
  o->reps = 3;
  o->progress_every = 0;
  o->ensemble = 1;
  return ADHA_OK;
}

adha_status adha_costmodel_train(adha_ctx *ctx, const adha_train_opts *o, adha_train_report *rep) {
  if (!ctx || !o) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (o->n_samples < 10 || o->batch == 0 || o->epochs == 0) return fail(ADHA_ERR_INVALID, "bad training options");
  if (o->ensemble > kMaxEnsemble) return fail(ADHA_ERR_INVALID, "at most %u networks", kMaxEnsemble);
  if (o->min_log2_n < 1 || o->max_log2_n > 26 || o->min_log2_n > o->max_log2_n)
    return fail(ADHA_ERR_INVALID, "record-count range must lie in [2^1, 2^26]");
  DeviceGuard guard(ctx->c.device);
  Ctx *c = &ctx->c;
  hipStream_t st = nullptr;
  ADHA_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } sg{st};
  auto t0 = std::chrono::steady_clock::now();
  Rng g{o->seed * 0x9E3779B97F4A7C15ull};
  const int64_t nmax = int64_t(1) << o->max_log2_n;
  const Shape big = training_shape(nmax);
  const uint64_t bufb = layout_aos(big, 64).nbytes + (uint64_t)64 * big.nfields() * 8;
  void *buf = nullptr, *idx = nullptr;
  ADHA_HIP(hipMalloc(&buf, bufb));
  hipError_t he = hipMalloc(&idx, (size_t)nmax * ADHA_MAX_DEGREE * 4);
  if (he != hipSuccess) {
    (void)hipFree(buf);
    return fail(ADHA_ERR_OOM, "training index buffer");
  }
  (void)hipMemsetAsync(buf, 0, bufb, st);
  adha_status rs = fill_uniform_index((int32_t *)idx, (uint64_t)nmax * ADHA_MAX_DEGREE, nmax, o->seed, st);
  std::vector<float> X, Y;
  hipEvent_t ea, eb;
  (void)hipEventCreate(&ea);
  (void)hipEventCreate(&eb);
  for (uint32_t i = 0; i < o->n_samples && rs >= 0; ++i) {
    const int64_t n = int64_t(1) << (o->min_log2_n + (int)g.below(o->max_log2_n - o->min_log2_n + 1));
    // gather indices must lie in [0, n): draw them for this n (in place)
    const Shape sh = training_shape(n);
    SectionDesc sec = random_section(g, sh);
    LayoutDesc lay = random_layout(g, sh, sec);
    if (sec.degree) rs = fill_uniform_index((int32_t *)idx, (uint64_t)n * sec.degree, n, o->seed + i, st);
    std::vector<double> ts;
    for (uint32_t r = 0; r <= o->reps && rs >= 0; ++r) {
      (void)hipEventRecord(ea, st);
      rs = section_launch(c, sec, lay, buf, (const int32_t *)idx, st);
      (void)hipEventRecord(eb, st);
      (void)hipEventSynchronize(eb);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, ea, eb);
      if (r) ts.push_back(ms * 1000.0);
    }
    if (rs < 0) break;
    std::sort(ts.begin(), ts.end());
    float f[ADHA_N_FEATURES];
    section_features(sec, lay, f);
    X.insert(X.end(), f, f + ADHA_N_FEATURES);
    Y.push_back((float)(std::log(std::max(1e-3, ts[ts.size() / 2])) - std::log(analytic_section_us(sec, lay))));
    if (o->progress_every && (i + 1) % o->progress_every == 0)
      std::fprintf(stderr, "costmodel: timed %u of %u sections\n", i + 1, o->n_samples);
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  (void)hipStreamSynchronize(st);
  (void)hipFree(buf);
  (void)hipFree(idx);
  if (rs < 0) return rs;
  auto t1 = std::chrono::steady_clock::now();

  // 90 / 10 split, then Adam on mini-batches, all on the device.
  const uint32_t ns = (uint32_t)Y.size(), nval = std::max<uint32_t>(1, ns / 10), ntr = ns - nval;
  const uint32_t B = std::min(o->batch, ntr);
  const uint32_t K = std::max<uint32_t>(1, o->ensemble);
  std::vector<float> P(ADHA_MLP_PARAMS, 0.0f), all;  // all: the K trained networks
  auto init = [&] {
    // He-uniform initial weights, zero biases (each network its own draw)
    std::fill(P.begin(), P.end(), 0.0f);
    const int fan[4] = {ADHA_N_FEATURES, 64, 64, 64}, outs[4] = {64, 64, 64, 1};
    size_t at = 0;
    for (int l = 0; l < 4; ++l) {
      const double lim = std::sqrt(6.0 / fan[l]);
      for (int q = 0; q < fan[l] * outs[l]; ++q) P[at + q] = (float)(lim * (2.0 * g.unit() - 1.0));
      at += (size_t)fan[l] * outs[l] + outs[l];
    }
  };
  float *dP = nullptr, *dG = nullptr, *dM = nullptr, *dV = nullptr, *dX = nullptr, *dY = nullptr, *dS = nullptr,
        *dL = nullptr;
  // scratch for the largest batch any call below uses: the mini-batches (B),
  // the whole training set (train loss) and the validation set
  const size_t scratch_floats = mlp_scratch_floats(std::max(std::max(B, nval), ntr));
  size_t need[8] = {ADHA_MLP_PARAMS, ADHA_MLP_PARAMS, ADHA_MLP_PARAMS, ADHA_MLP_PARAMS, X.size(), Y.size(),
                    scratch_floats, 4};
  float **ptrs[8] = {&dP, &dG, &dM, &dV, &dX, &dY, &dS, &dL};
  adha_status result = ADHA_OK;
  for (int q = 0; q < 8; ++q)
    if (hipMalloc((void **)ptrs[q], need[q] * 4) != hipSuccess) result = fail(ADHA_ERR_OOM, "training buffers");
  if (result >= 0) {
    (void)hipMemcpy(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice);
    (void)hipMemcpy(dY, Y.data(), Y.size() * 4, hipMemcpyHostToDevice);
  }
  // every network on the same data, from its own initial weights; the
  // validation figures are those of their mean prediction
  std::vector<double> pred_sum(nval, 0.0);
  double tl_sum = 0.0;
  for (uint32_t k = 0; k < K && result >= 0; ++k) {
    init();
    (void)hipMemcpy(dP, P.data(), P.size() * 4, hipMemcpyHostToDevice);
    (void)hipMemset(dM, 0, ADHA_MLP_PARAMS * 4);
    (void)hipMemset(dV, 0, ADHA_MLP_PARAMS * 4);
    uint32_t step = 0;
    for (uint32_t ep = 0; ep < o->epochs && result >= 0; ++ep) {
      // the step size decays along a half cosine, from lr to lr / 20
      const float lr = (float)(o->lr * (0.05 + 0.95 * 0.5 * (1.0 + std::cos(3.141592653589793 * ep / o->epochs))));
      for (uint32_t b0 = 0; b0 + B <= ntr && result >= 0; b0 += B) {
        result = mlp_backward(c, dP, dX + (size_t)b0 * ADHA_N_FEATURES, dY + b0, B, dG, dL, dS, scratch_floats, st);
        if (result >= 0) result = mlp_adam(c, dP, dG, dM, dV, lr, 0.9f, 0.999f, 1e-8f, ++step, st);
      }
    }
    float tl = 0.f;
    if (result >= 0) {
      result = mlp_backward(c, dP, dX, dY, ntr, dG, dL, dS, scratch_floats, st);
      (void)hipStreamSynchronize(st);
      (void)hipMemcpy(&tl, dL, 4, hipMemcpyDeviceToHost);
      tl_sum += tl;
    }
    std::vector<float> pred(nval);
    if (result >= 0) {
      result = mlp_forward(c, dP, dX + (size_t)ntr * ADHA_N_FEATURES, nval, dS, st);
      (void)hipStreamSynchronize(st);
      (void)hipMemcpy(pred.data(), dS, nval * 4, hipMemcpyDeviceToHost);
      (void)hipMemcpy(P.data(), dP, P.size() * 4, hipMemcpyDeviceToHost);
      for (uint32_t q = 0; q < nval; ++q) pred_sum[q] += pred[q];
      all.insert(all.end(), P.begin(), P.end());
    }
  }
  if (result >= 0) {
    {
      double mse = 0, mape = 0;
      for (uint32_t q = 0; q < nval; ++q) {
        const double pm = pred_sum[q] / K;
        const double d = pm - Y[ntr + q];
        mse += d * d;
        mape += std::fabs(std::exp(pm - Y[ntr + q]) - 1.0);
      }
      const double tl = tl_sum / K;
      c->model = all;
      c->n_models = K;
      c->has_model = true;
      c->mlp_params_ok = false;
      if (rep) {
        rep->gen_seconds = std::chrono::duration<double>(t1 - t0).count();
        rep->train_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
        rep->train_loss = tl;
        rep->val_loss = mse / nval;
        rep->val_mape = mape / nval;
        rep->n_train = ntr;
        rep->n_val = nval;
      }
    }
  }
  for (int q = 0; q < 8; ++q)
    if (*ptrs[q]) (void)hipFree(*ptrs[q]);
  return result;
}

adha_status adha_costmodel_save(const adha_ctx *ctx, const char *path) {
  if (!ctx || !path) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!ctx->c.has_model) return fail(ADHA_ERR_STATE, "no cost model to save");
  FILE *f = fopen(path, "wb");
  if (!f) return fail(ADHA_ERR_IO, "cannot open %s for writing", path);
  const char magic[8] = {'A', 'D', 'H', 'A', 'M', 'L', 'P', '3'};
  const uint32_t k = ctx->c.n_models, n = ADHA_MLP_PARAMS;
  const size_t total = (size_t)k * n;
  const uint64_t h = fnv1a(ctx->c.model.data(), total * 4);
  bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&k, 4, 1, f) == 1 && fwrite(&n, 4, 1, f) == 1 &&
            fwrite(ctx->c.model.data(), 4, total, f) == total && fwrite(&h, 8, 1, f) == 1;
  ok = (fclose(f) == 0) && ok;
  if (!ok) return fail(ADHA_ERR_IO, "write to %s failed", path);
  return ADHA_OK;
}

adha_status adha_costmodel_load(adha_ctx *ctx, const char *path) {
  if (!ctx || !path) return fail(ADHA_ERR_INVALID, "NULL argument");
  ctx->c.has_model = false;
  ctx->c.model.clear();
  ctx->c.mlp_params_ok = false;
  FILE *f = fopen(path, "rb");
  if (!f) return fail(ADHA_ERR_IO, "cannot open %s", path);
  char magic[8];
  uint32_t k = 0, n = 0;
  uint64_t h = 0;
  std::vector<float> P;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "ADHAMLP3", 8) == 0 && fread(&k, 4, 1, f) == 1 &&
            k >= 1 && k <= kMaxEnsemble && fread(&n, 4, 1, f) == 1 && n == ADHA_MLP_PARAMS;
  if (ok) {
    P.resize((size_t)k * n);
    ok = fread(P.data(), 4, P.size(), f) == P.size() && fread(&h, 8, 1, f) == 1;
  }
  fclose(f);
  if (!ok) return fail(ADHA_ERR_IO, "%s is not a cost-model file (short or bad header)", path);
  if (fnv1a(P.data(), P.size() * 4) != h) return fail(ADHA_ERR_IO, "%s failed its checksum", path);
  ctx->c.model = P;
  ctx->c.n_models = k;
  ctx->c.has_model = true;
  ctx->c.mlp_params_ok = false;
  return ADHA_OK;
}

adha_status adha_costmodel_predict(adha_ctx *ctx, const adha_section *sec, const adha_layout *l, double *us) {
  if (!ctx || !sec || !l || !us) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!sec->d.shape.same(l->d.shape)) return fail(ADHA_ERR_INVALID, "section and layout describe different structs");
  DeviceGuard g(ctx->c.device);
  std::vector<std::vector<float>> feats(1, std::vector<float>(ADHA_N_FEATURES));
  section_features(sec->d, l->d, feats[0].data());
  std::vector<double> out;
  ADHA_TRY(predict_costs(&ctx->c, feats, {analytic_section_us(sec->d, l->d)}, &out, nullptr));
  *us = out[0];
  return ADHA_OK;
}

}  // extern "C"
