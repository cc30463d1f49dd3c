// Autotuner for the remap launches and its persistent database.
//
// A remap is bound by HBM bandwidth, and how close it gets depends on the
// tile size, how many workgroups share a compute unit, the order in which
// workgroups walk the tiles and whether accesses are marked as streaming.
// The tuner times a grid of these on the caller's buffers and keeps the
// fastest, per layout-pair class (single remaps) or as the batch policy.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "adha_impl.h"

namespace adha {

template <class Fn>
static adha_status median_us(hipStream_t stream, uint32_t reps, Fn fn, double *out) {
  hipEvent_t a, b;
  ADHA_HIP(hipEventCreate(&a));
  ADHA_HIP(hipEventCreate(&b));
  std::vector<double> ts;
  adha_status st = fn();  // warm-up (also builds the launch descriptor)
  for (uint32_t r = 0; r < reps && st >= 0; ++r) {
    (void)hipEventRecord(a, stream);
    st = fn();
    (void)hipEventRecord(b, stream);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    ts.push_back(ms * 1000.0);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st < 0) return st;
  std::sort(ts.begin(), ts.end());
  *out = ts.empty() ? 0.0 : ts[ts.size() / 2];
  return ADHA_OK;
}

static const uint32_t kTileBytes[] = {4096, 8192, 16384, 32768};
static const uint32_t kWgPerCu[] = {1, 2, 4, 8, 16, 32};
// A batch mixes arrays whose tiles hold different byte counts; more
// workgroups than fit at once let the ones that finish early take the rest,
// so the batch policy also tries 64 per CU.
static const uint32_t kBatchWgPerCu[] = {1, 2, 4, 8, 16, 32, 64};

static void to_abi(const TileShape &s, adha_tile_shape *o) {
  o->tile_records = s.R;
  o->slots = s.K;
  o->pad_shift = s.shift;
  o->wg_per_cu = s.wg_per_cu;
  o->order = s.strided + 1;
  o->nontemporal = s.nt + 1;
}

static uint64_t fnv1a(const std::string &s) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : s) h = (h ^ c) * 1099511628211ull;
  return h;
}

}  // namespace adha

using namespace adha;

extern "C" {

adha_status adha_tune_remap(adha_ctx *ctx, const adha_layout *src_l, const void *src, uint64_t src_cap,
                            const adha_layout *dst_l, void *dst, uint64_t dst_cap, uint32_t reps, void *stream,
                            adha_tile_shape *best, double *best_us, double *default_us) {
  if (!ctx || !best || !best_us || !default_us) return fail(ADHA_ERR_INVALID, "NULL argument");
  ADHA_TRY(validate_remap(src_l, src, src_cap, dst_l, dst, dst_cap));
  if (src_l->d.shape.n == 0) return fail(ADHA_ERR_INVALID, "nothing to tune on an empty struct");
  DeviceGuard g(ctx->c.device);
  Ctx *c = &ctx->c;
  hipStream_t st = (hipStream_t)stream;
  reps = std::max<uint32_t>(1, reps);
  TileShape def;
  ADHA_TRY(policy_shape(src_l->d, dst_l->d, default_tile_bytes(src_l->d), 4, 1, 1, &def));
  if (def.R == 0) return fail(ADHA_ERR_UNSUPPORTED, "records too large for a tiled remap");
  double t_def = 0;
  ADHA_TRY(median_us(st, reps, [&] { return remap_with_shape(c, src_l, src, dst_l, dst, def, st); }, &t_def));
  TileShape bs = def;
  double bt = t_def;
  for (uint32_t tb : kTileBytes)
    for (uint32_t wg : kWgPerCu)
      for (uint32_t order = 0; order < 2; ++order)
        for (uint32_t nt = 0; nt < 2; ++nt) {
          TileShape s;
          ADHA_TRY(policy_shape(src_l->d, dst_l->d, tb, wg, order, nt, &s));
          if (s.R == 0 || check_shape(src_l->d, dst_l->d, s) < 0) continue;
          double t = 0;
          ADHA_TRY(median_us(st, reps, [&] { return remap_with_shape(c, src_l, src, dst_l, dst, s, st); }, &t));
          if (t < bt) {
            bt = t;
            bs = s;
          }
        }
  clear_error();
  c->forced_shapes[{src_l->id, dst_l->id}] = bs;
  c->tunedb[tune_key(src_l->d, dst_l->d)] = bs;
  to_abi(bs, best);
  *best_us = bt;
  *default_us = t_def;
  return ADHA_OK;
}

adha_status adha_tune_batched(adha_ctx *ctx, uint32_t n, const adha_remap_item *items, uint32_t reps, void *stream,
                              uint32_t *tile_bytes, adha_tile_shape *best, double *best_us, double *default_us) {
  if (!ctx || !items || !tile_bytes || !best || !best_us || !default_us) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (n == 0) return fail(ADHA_ERR_INVALID, "no items");
  for (uint32_t i = 0; i < n; ++i) {
    const adha_remap_item &it = items[i];
    adha_status s = validate_remap(it.src_layout, it.src, it.src_cap, it.dst_layout, it.dst, it.dst_cap);
    if (s < 0) return s;
  }
  ADHA_TRY(check_items_disjoint(n, items));
  DeviceGuard g(ctx->c.device);
  Ctx *c = &ctx->c;
  hipStream_t st = (hipStream_t)stream;
  reps = std::max<uint32_t>(1, reps);
  const Ctx::BatchPolicy saved = c->batch;
  double t_def = 0;
  c->batch = Ctx::BatchPolicy();
  ADHA_TRY(median_us(st, reps, [&] { return batch_run(c, n, items, 0, st); }, &t_def));
  Ctx::BatchPolicy bp = c->batch;
  double bt = t_def;
  for (uint32_t tb : kTileBytes)
    for (uint32_t wg : kBatchWgPerCu)
      for (uint32_t order = 0; order < 2; ++order)
        for (uint32_t nt = 0; nt < 2; ++nt) {
          c->batch.tile_bytes = tb;
          c->batch.wg_per_cu = wg;
          c->batch.strided = order;
          c->batch.nt = nt;
          double t = 0;
          adha_status s = median_us(st, reps, [&] { return batch_run(c, n, items, 0, st); }, &t);
          if (s < 0) {
            c->batch = saved;
            return s;
          }
          if (t < bt) {
            bt = t;
            bp = c->batch;
          }
        }
  c->batch = bp;
  *tile_bytes = bp.tile_bytes;
  TileShape shown;
  shown.R = 0;
  shown.K = 0;
  shown.shift = 6;
  shown.wg_per_cu = bp.wg_per_cu;
  shown.strided = bp.strided;
  shown.nt = bp.nt;
  to_abi(shown, best);
  *best_us = bt;
  *default_us = t_def;
  return ADHA_OK;
}

adha_status adha_tune_save(const adha_ctx *ctx, const char *path) {
  if (!ctx || !path) return fail(ADHA_ERR_INVALID, "NULL argument");
  std::string body = "ADHA-TUNE 1\n";
  char line[256];
  snprintf(line, sizeof line, "batch %u %u %u %u\n", ctx->c.batch.tile_bytes, ctx->c.batch.wg_per_cu,
           ctx->c.batch.strided, ctx->c.batch.nt);
  body += line;
  for (auto &kv : ctx->c.tunedb) {
    const TileShape &s = kv.second;
    snprintf(line, sizeof line, "%s %u %u %u %u %u %u\n", kv.first.c_str(), s.R, s.K, s.shift, s.wg_per_cu,
             s.strided, s.nt);
    body += line;
  }
  snprintf(line, sizeof line, "checksum %016llx\n", (unsigned long long)fnv1a(body));
  FILE *f = fopen(path, "w");
  if (!f) return fail(ADHA_ERR_IO, "cannot open %s for writing", path);
  bool ok = fputs(body.c_str(), f) >= 0 && fputs(line, f) >= 0;
  ok = (fclose(f) == 0) && ok;
  if (!ok) return fail(ADHA_ERR_IO, "write to %s failed", path);
  return ADHA_OK;
}

adha_status adha_tune_load(adha_ctx *ctx, const char *path) {
  if (!ctx || !path) return fail(ADHA_ERR_INVALID, "NULL argument");
  FILE *f = fopen(path, "r");
  if (!f) return fail(ADHA_ERR_IO, "cannot open %s", path);
  std::vector<std::string> lines;
  char buf[512];
  while (fgets(buf, sizeof buf, f)) lines.push_back(buf);
  fclose(f);
  if (lines.size() < 3 || lines[0] != "ADHA-TUNE 1\n") return fail(ADHA_ERR_IO, "%s is not a tuning file", path);
  std::string body;
  for (size_t i = 0; i + 1 < lines.size(); ++i) body += lines[i];
  unsigned long long sum = 0;
  if (sscanf(lines.back().c_str(), "checksum %llx", &sum) != 1 || sum != fnv1a(body))
    return fail(ADHA_ERR_IO, "%s failed its checksum", path);
  Ctx::BatchPolicy bp;
  if (sscanf(lines[1].c_str(), "batch %u %u %u %u", &bp.tile_bytes, &bp.wg_per_cu, &bp.strided, &bp.nt) != 4 ||
      bp.wg_per_cu == 0 || bp.wg_per_cu > 64 || bp.strided > 1 || bp.nt > 1)
    return fail(ADHA_ERR_IO, "%s: bad batch line", path);
  std::map<std::string, TileShape> db;
  for (size_t i = 2; i + 1 < lines.size(); ++i) {
    char key[256];
    TileShape s;
    if (sscanf(lines[i].c_str(), "%255s %u %u %u %u %u %u", key, &s.R, &s.K, &s.shift, &s.wg_per_cu, &s.strided,
               &s.nt) != 7)
      return fail(ADHA_ERR_IO, "%s: bad line %zu", path, i + 1);
    db[key] = s;
  }
  ctx->c.batch = bp;
  ctx->c.tunedb = db;
  return ADHA_OK;
}

}  // extern "C"
