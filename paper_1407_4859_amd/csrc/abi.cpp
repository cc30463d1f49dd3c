// The exported C-ABI: argument validation on the host, then dispatch.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>

#include "adha_impl.h"

namespace adha {
const char *last_error();

Ctx::~Ctx() {
  for (auto &g : graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  for (auto &kv : remap_cache)
    if (kv.second.dev) (void)hipFree(kv.second.dev);
  if (err_flag) (void)hipFree(err_flag);
  if (reduce_partials) (void)hipFree(reduce_partials);
  for (float *q : {mlp_params, mlp_x, mlp_y})
    if (q) (void)hipFree(q);
}

adha_status ctx_reduce_scratch(Ctx *ctx) {
  if (ctx->reduce_partials) return ADHA_OK;
  if (hipMalloc(&ctx->reduce_partials, kReducePartialPairs * 16) != hipSuccess) {
    ctx->reduce_partials = nullptr;
    return fail(ADHA_ERR_OOM, "reduction scratch of %llu bytes failed", (unsigned long long)(kReducePartialPairs * 16));
  }
  return ADHA_OK;
}

static bool aligned(const void *p) { return ((uintptr_t)p & 255u) == 0; }

static adha_status check_dev_buf(const char *what, const void *p, uint64_t cap, uint64_t need) {
  if (need == 0) return ADHA_OK;
  if (!p) return fail(ADHA_ERR_INVALID, "%s is NULL", what);
  if (!aligned(p)) return fail(ADHA_ERR_INVALID, "%s is not 256-byte aligned", what);
  if (cap < need)
    return fail(ADHA_ERR_INVALID, "%s holds %llu bytes, the layout needs %llu", what,
                (unsigned long long)cap, (unsigned long long)need);
  return ADHA_OK;
}

static bool overlap(const void *a, uint64_t na, const void *b, uint64_t nb) {
  if (!na || !nb) return false;
  uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

// No item's destination may overlap another item's destination or source
// (an item's own source and destination were checked on their own).  Sorted
// sweeps instead of all pairs: destinations by start with the running end,
// then each destination against the sources that start before its end,
// through the running maximum of their ends.
adha_status check_items_disjoint(uint32_t n, const adha_remap_item *items) {
  struct Iv {
    uintptr_t lo, hi;
    uint32_t item;
  };
  std::vector<Iv> d, s;
  d.reserve(n);
  s.reserve(n);
  for (uint32_t i = 0; i < n; ++i) {
    const uint64_t dn = items[i].dst_layout->d.nbytes, sn = items[i].src_layout->d.nbytes;
    if (dn) d.push_back({(uintptr_t)items[i].dst, (uintptr_t)items[i].dst + dn, i});
    if (sn) s.push_back({(uintptr_t)items[i].src, (uintptr_t)items[i].src + sn, i});
  }
  auto by_lo = [](const Iv &a, const Iv &b) { return a.lo < b.lo; };
  std::sort(d.begin(), d.end(), by_lo);
  std::sort(s.begin(), s.end(), by_lo);
  auto report = [](uint32_t a, uint32_t b) {
    return fail(ADHA_ERR_INVALID, "items %u and %u overlap", std::min(a, b), std::max(a, b));
  };
  for (size_t k = 1, top = 0; k < d.size(); ++k) {
    if (d[k].lo < d[top].hi) return report(d[top].item, d[k].item);
    if (d[k].hi > d[top].hi) top = k;
  }
  std::vector<size_t> best(s.size());  // index of the largest end among s[0..k]
  for (size_t k = 0; k < s.size(); ++k) best[k] = k && s[best[k - 1]].hi >= s[k].hi ? best[k - 1] : k;
  for (const Iv &x : d) {
    const size_t c = std::lower_bound(s.begin(), s.end(), Iv{x.hi, 0, 0}, by_lo) - s.begin();
    if (c && s[best[c - 1]].hi > x.lo) return report(s[best[c - 1]].item, x.item);
  }
  return ADHA_OK;
}

static const size_t kCacheLimit = 4096;

// Drops every cached descriptor blob and every graph that launches them.
static adha_status flush_cache(Ctx *ctx) {
  ADHA_HIP(hipDeviceSynchronize());
  for (auto &ge : ctx->graphs) {
    if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
    if (ge.graph) (void)hipGraphDestroy(ge.graph);
  }
  ctx->graphs.clear();
  for (auto &kv : ctx->remap_cache) (void)hipFree(kv.second.dev);
  ctx->remap_cache.clear();
  return ADHA_OK;
}

// Cached remap launch for one (src layout, dst layout, shape); pointers are
// passed at run time.
adha_status prepared_for(Ctx *ctx, const adha_layout *a, const adha_layout *b,
                                const TileShape &sh, const RemapPrepared **out) {
  std::vector<uint64_t> key{1, a->id, b->id, sh.R, sh.K, sh.shift, sh.wg_per_cu, sh.strided, sh.nt};
  auto it = ctx->remap_cache.find(key);
  if (it == ctx->remap_cache.end()) {
    if (ctx->remap_cache.size() >= kCacheLimit) ADHA_TRY(flush_cache(ctx));
    RemapPrepared p;
    ADHA_TRY(remap_prepare(ctx, {&a->d}, {nullptr}, {&b->d}, {nullptr}, {sh}, &p));
    it = ctx->remap_cache.emplace(key, p).first;
  }
  *out = &it->second;
  return ADHA_OK;
}

adha_status shape_for(Ctx *ctx, const adha_layout *a, const adha_layout *b, TileShape *sh) {
  auto it = ctx->forced_shapes.find({a->id, b->id});
  if (it != ctx->forced_shapes.end()) {
    *sh = it->second;
    return ADHA_OK;
  }
  return choose_shape(ctx, a->d, b->d, sh);
}

// Shape of one array inside a batched launch: the context's batch policy
// (tile bytes, workgroups per CU, order, streaming) unless the pair was forced.
static adha_status batch_shape_for(Ctx *ctx, const adha_layout *a, const adha_layout *b, TileShape *sh) {
  auto it = ctx->forced_shapes.find({a->id, b->id});
  if (it != ctx->forced_shapes.end()) {
    *sh = it->second;
    return ADHA_OK;
  }
  return policy_shape(a->d, b->d, ctx->batch.tile_bytes, ctx->batch.wg_per_cu, ctx->batch.strided,
                      ctx->batch.nt, sh);
}

adha_status remap_with_shape(Ctx *ctx, const adha_layout *sl, const void *src, const adha_layout *dl,
                             void *dst, const TileShape &sh, hipStream_t stream) {
  if (sl->d.shape.n == 0 || dl->d.nbytes == 0) return ADHA_OK;
  const RemapPrepared *p = nullptr;
  ADHA_TRY(prepared_for(ctx, sl, dl, sh, &p));
  return remap_run(ctx, *p, src, dst, stream);
}

adha_status validate_remap(const adha_layout *sl, const void *src, uint64_t src_cap,
                                  const adha_layout *dl, const void *dst, uint64_t dst_cap) {
  if (!sl || !dl) return fail(ADHA_ERR_INVALID, "layout is NULL");
  if (!sl->d.shape.same(dl->d.shape))
    return fail(ADHA_ERR_INVALID, "source and destination layouts describe different structs");
  ADHA_TRY(check_dev_buf("src", src, src_cap, sl->d.nbytes));
  ADHA_TRY(check_dev_buf("dst", dst, dst_cap, dl->d.nbytes));
  if (overlap(src, sl->d.nbytes, dst, dl->d.nbytes))
    return fail(ADHA_ERR_INVALID, "src and dst overlap (remaps are out of place)");
  return ADHA_OK;
}

// A layout's content (shape, groups, tiles, bases) as key words.
static void content_key(const LayoutDesc &L, std::vector<uint64_t> *k) {
  k->push_back((uint64_t)L.shape.n);
  k->push_back((uint64_t)L.shape.nfields());
  for (int f = 0; f < L.shape.nfields(); ++f) k->push_back(((uint64_t)L.shape.dtype[f] << 32) | L.shape.ebytes[f]);
  k->push_back(L.groups.size());
  for (const Group &g : L.groups) {
    k->push_back(((uint64_t)g.T << 32) | g.fields.size());
    k->push_back(g.base);
    for (int f : g.fields) k->push_back((uint64_t)f);
  }
}

// The moving part of an in-place remap src -> dst inside one buffer, run
// with a descriptor cached by the layouts' content (the same pairs recur
// every time a plan runs).
adha_status remap_in_place(Ctx *ctx, const LayoutDesc &src, const LayoutDesc &dst, void *buf, hipStream_t stream) {
  LayoutDesc a, b;
  bool moves = false;
  ADHA_TRY(in_place_parts(src, dst, &a, &b, &moves));
  if (!moves || a.shape.n == 0) return ADHA_OK;
  TileShape sh;
  ADHA_TRY(choose_shape(ctx, a, b, &sh));
  std::vector<uint64_t> key{3, sh.R, sh.K, sh.shift, sh.wg_per_cu, sh.strided, sh.nt};
  content_key(a, &key);
  content_key(b, &key);
  auto it = ctx->remap_cache.find(key);
  if (it == ctx->remap_cache.end()) {
    if (ctx->remap_cache.size() >= kCacheLimit) ADHA_TRY(flush_cache(ctx));
    RemapPrepared p;
    ADHA_TRY(remap_prepare(ctx, {&a}, {nullptr}, {&b}, {nullptr}, {sh}, &p));
    it = ctx->remap_cache.emplace(key, p).first;
  }
  return remap_run(ctx, it->second, buf, buf, stream);
}

adha_status remap_one(Ctx *ctx, const adha_layout *sl, const void *src, const adha_layout *dl,
                      void *dst, hipStream_t stream) {
  if (sl->d.shape.n == 0 || dl->d.nbytes == 0) return ADHA_OK;
  TileShape sh;
  ADHA_TRY(shape_for(ctx, sl, dl, &sh));
  const RemapPrepared *p = nullptr;
  ADHA_TRY(prepared_for(ctx, sl, dl, sh, &p));
  return remap_run(ctx, *p, src, dst, stream);
}

}  // namespace adha

using namespace adha;

extern "C" {

const char *adha_status_string(adha_status st) {
  switch (st) {
    case ADHA_OK: return "ok";
    case ADHA_WARN_FALLBACK: return "ok (fallback taken)";
    case ADHA_ERR_INVALID: return "invalid argument";
    case ADHA_ERR_OOM: return "out of memory";
    case ADHA_ERR_DEVICE: return "device error";
    case ADHA_ERR_STATE: return "invalid state";
    case ADHA_ERR_UNSUPPORTED: return "unsupported";
    case ADHA_ERR_IO: return "i/o error";
    default: return "unknown status";
  }
}

const char *adha_last_error(void) { return adha::last_error(); }

int32_t adha_version(void) { return 10000; }

// ------------------------------------------------------------------ context
adha_status adha_ctx_create(int32_t device, adha_ctx **out) {
  if (!out) return fail(ADHA_ERR_INVALID, "out is NULL");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(ADHA_ERR_DEVICE, "no HIP device visible");
  if (device < 0 || device >= n) return fail(ADHA_ERR_INVALID, "device %d not in [0, %d)", device, n);
  hipDeviceProp_t prop;
  ADHA_HIP(hipGetDeviceProperties(&prop, device));
  std::string arch = prop.gcnArchName;
  if (arch.compare(0, 6, "gfx950") != 0)
    return fail(ADHA_ERR_DEVICE, "device %d is %s; this library is built for gfx950", device, arch.c_str());
  auto *c = new (std::nothrow) adha_ctx;
  if (!c) return fail(ADHA_ERR_OOM, "context allocation failed");
  c->c.device = device;
  c->c.arch = arch;
  c->c.cu_count = prop.multiProcessorCount;
  DeviceGuard g(device);
  if (hipMalloc((void **)&c->c.err_flag, 256) != hipSuccess ||
      hipMemset(c->c.err_flag, 0, 256) != hipSuccess) {
    delete c;
    return fail(ADHA_ERR_OOM, "context scratch allocation failed");
  }
  const adha_status ss = static_scratch_address(device, &c->c.static_scratch);
  if (ss < 0) {
    delete c;
    return ss;
  }
  *out = c;
  return ADHA_OK;
}

adha_status adha_ctx_destroy(adha_ctx *ctx) {
  if (!ctx) return ADHA_OK;
  DeviceGuard g(ctx->c.device);
  (void)hipDeviceSynchronize();
  delete ctx;
  return ADHA_OK;
}

adha_status adha_ctx_check(adha_ctx *ctx, void *stream) {
  if (!ctx) return fail(ADHA_ERR_INVALID, "ctx is NULL");
  DeviceGuard g(ctx->c.device);
  ADHA_HIP(hipStreamSynchronize((hipStream_t)stream));
  uint32_t flag = 0;
  ADHA_HIP(hipMemcpy(&flag, ctx->c.err_flag, 4, hipMemcpyDeviceToHost));
  if (ctx->c.host_bad) {
    flag = 1;
    ctx->c.host_bad = 0;
  }
  if (flag) {
    ADHA_HIP(hipMemset(ctx->c.err_flag, 0, 4));
    return fail(ADHA_ERR_INVALID,
                "a gather met an index outside [0, N) or a reduction a key outside [0, n_keys); "
                "those terms or records were left out");
  }
  return ADHA_OK;
}

adha_status adha_ctx_cu_count(const adha_ctx *ctx, int32_t *out) {
  if (!ctx || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  *out = ctx->c.cu_count;
  return ADHA_OK;
}

adha_status adha_ctx_set_option(adha_ctx *ctx, adha_option opt, int64_t value) {
  if (!ctx) return fail(ADHA_ERR_INVALID, "ctx is NULL");
  switch (enum_value(opt)) {
    case ADHA_OPT_SPAN_GATHER:
      if (value != 0 && value != 1) return fail(ADHA_ERR_INVALID, "span-gather option is 0 or 1");
      ctx->c.no_span = value == 0;
      return ADHA_OK;
    case ADHA_OPT_REDUCE_WG_PER_CU:
      if (value < 1 || value > 32) return fail(ADHA_ERR_INVALID, "workgroups per CU %lld not in [1, 32]", (long long)value);
      ctx->c.reduce_wg_per_cu = (uint32_t)value;
      return ADHA_OK;
    case ADHA_OPT_HOST_THREADS:
      if (value < 0 || value > 256) return fail(ADHA_ERR_INVALID, "host threads %lld not in [0, 256]", (long long)value);
      ctx->c.host_threads = (uint32_t)value;
      return ADHA_OK;
    case ADHA_OPT_REDUCE_COMPENSATED:
      if (value != 0 && value != 1) return fail(ADHA_ERR_INVALID, "compensated-reduction option is 0 or 1");
      ctx->c.reduce_plain = value == 0;
      return ADHA_OK;
    default:
      return fail(ADHA_ERR_INVALID, "unknown option %d", enum_value(opt));
  }
}

// ------------------------------------------------------------------ struct
adha_status adha_struct_create(int64_t n_records, adha_struct **out) {
  if (!out) return fail(ADHA_ERR_INVALID, "out is NULL");
  if (n_records < 0 || n_records > (int64_t(1) << 40))
    return fail(ADHA_ERR_INVALID, "n_records %lld not in [0, 2^40]", (long long)n_records);
  auto *s = new (std::nothrow) adha_struct;
  if (!s) return fail(ADHA_ERR_OOM, "struct allocation failed");
  s->shape.n = n_records;
  *out = s;
  return ADHA_OK;
}

adha_status adha_struct_add_field(adha_struct *s, adha_dtype dt, uint32_t elem_bytes, int32_t *out_id) {
  if (!s) return fail(ADHA_ERR_INVALID, "struct is NULL");
  switch (enum_value(dt)) {
    case ADHA_F32:
    case ADHA_I32:
    case ADHA_U32:
      if (elem_bytes != 4) return fail(ADHA_ERR_INVALID, "F32 / I32 / U32 fields have 4-byte elements");
      break;
    case ADHA_U16:
    case ADHA_I16:
      if (elem_bytes != 2) return fail(ADHA_ERR_INVALID, "U16 / I16 fields have 2-byte elements");
      break;
    case ADHA_U8:
      if (elem_bytes != 1) return fail(ADHA_ERR_INVALID, "U8 fields have 1-byte elements");
      break;
    case ADHA_F64:
      if (elem_bytes != 8) return fail(ADHA_ERR_INVALID, "F64 fields have 8-byte elements");
      break;
    case ADHA_RAW:
      if (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8)
        return fail(ADHA_ERR_INVALID, "RAW element size %u not in {1, 2, 4, 8}", elem_bytes);
      break;
    default:
      return fail(ADHA_ERR_INVALID, "unknown dtype %d", enum_value(dt));
  }
  if (s->shape.nfields() >= ADHA_MAX_FIELDS) return fail(ADHA_ERR_INVALID, "at most %d fields", ADHA_MAX_FIELDS);
  if (s->shape.record_bytes() + elem_bytes > 2048) return fail(ADHA_ERR_INVALID, "records are limited to 2048 bytes");
  if ((uint64_t)(s->shape.record_bytes() + elem_bytes) * (uint64_t)s->shape.n > (uint64_t(1) << 46))
    return fail(ADHA_ERR_INVALID, "N * record bytes exceeds 2^46");
  s->shape.dtype.push_back((int32_t)dt);
  s->shape.ebytes.push_back(elem_bytes);
  if (out_id) *out_id = s->shape.nfields() - 1;
  return ADHA_OK;
}

adha_status adha_struct_destroy(adha_struct *s) {
  delete s;
  return ADHA_OK;
}

adha_status adha_struct_info(const adha_struct *s, int64_t *n_records, int32_t *n_fields,
                             uint32_t *record_bytes) {
  if (!s) return fail(ADHA_ERR_INVALID, "struct is NULL");
  if (n_records) *n_records = s->shape.n;
  if (n_fields) *n_fields = s->shape.nfields();
  if (record_bytes) *record_bytes = s->shape.record_bytes();
  return ADHA_OK;
}

// ------------------------------------------------------------------ layouts
static adha_status emit_layout(LayoutDesc d, adha_layout **out) {
  adha_layout *l = new_layout(std::move(d));
  if (!l) return fail(ADHA_ERR_OOM, "layout allocation failed");
  *out = l;
  return ADHA_OK;
}

adha_status adha_layout_create(const adha_struct *s, uint32_t n_groups, const uint32_t *group_of_field,
                               const uint32_t *tile_of_group, adha_layout **out) {
  if (!s || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  LayoutDesc d;
  ADHA_TRY(build_layout(s->shape, n_groups, group_of_field, tile_of_group, &d));
  return emit_layout(std::move(d), out);
}

adha_status adha_layout_aos(const adha_struct *s, adha_layout **out) {
  if (!s || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (s->shape.nfields() == 0) return fail(ADHA_ERR_INVALID, "struct has no fields");
  return emit_layout(layout_aos(s->shape), out);
}

adha_status adha_layout_soa(const adha_struct *s, adha_layout **out) {
  if (!s || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (s->shape.nfields() == 0) return fail(ADHA_ERR_INVALID, "struct has no fields");
  return emit_layout(layout_soa(s->shape), out);
}

adha_status adha_layout_destroy(adha_layout *l) {
  delete l;
  return ADHA_OK;
}

adha_status adha_layout_nbytes(const adha_layout *l, uint64_t *out) {
  if (!l || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  *out = l->d.nbytes;
  return ADHA_OK;
}

adha_status adha_layout_addr(const adha_layout *l, int64_t r, int32_t f, uint64_t *out) {
  if (!l || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (r < 0 || r >= l->d.shape.n) return fail(ADHA_ERR_INVALID, "record %lld out of range", (long long)r);
  if (f < 0 || f >= l->d.shape.nfields()) return fail(ADHA_ERR_INVALID, "field %d out of range", f);
  *out = l->d.addr(r, f);
  return ADHA_OK;
}

adha_status adha_layout_groups(const adha_layout *l, uint32_t *n_groups, uint32_t *group_of_field,
                               uint32_t *tile_of_group) {
  if (!l) return fail(ADHA_ERR_INVALID, "layout is NULL");
  if (n_groups) *n_groups = (uint32_t)l->d.groups.size();
  if (group_of_field)
    for (int f = 0; f < l->d.shape.nfields(); ++f) group_of_field[f] = l->d.group_of[f];
  if (tile_of_group)
    for (size_t g = 0; g < l->d.groups.size(); ++g) tile_of_group[g] = l->d.groups[g].T;
  return ADHA_OK;
}

adha_status adha_layout_equal(const adha_layout *a, const adha_layout *b, int32_t *out) {
  if (!a || !b || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  *out = a->d.same_map(b->d) ? 1 : 0;
  return ADHA_OK;
}

adha_status adha_layout_place(const adha_layout *l, uint32_t n_groups, const uint64_t *bases, adha_layout **out) {
  if (!l || !out || (n_groups && !bases)) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (n_groups != l->d.groups.size())
    return fail(ADHA_ERR_INVALID, "%u bases given, the layout has %zu groups", n_groups, l->d.groups.size());
  LayoutDesc d = l->d;
  ADHA_TRY(place_layout(&d, std::vector<uint64_t>(bases, bases + n_groups)));
  adha_layout *p = new_layout(std::move(d));
  if (!p) return fail(ADHA_ERR_OOM, "layout allocation failed");
  *out = p;
  return ADHA_OK;
}

adha_status adha_layout_bases(const adha_layout *l, uint64_t *bases) {
  if (!l || !bases) return fail(ADHA_ERR_INVALID, "NULL argument");
  for (size_t g = 0; g < l->d.groups.size(); ++g) bases[g] = l->d.groups[g].base;
  return ADHA_OK;
}

// ------------------------------------------------------------------ remap
adha_status adha_remap(adha_ctx *ctx, const adha_layout *src_l, const void *src, uint64_t src_cap,
                       const adha_layout *dst_l, void *dst, uint64_t dst_cap, void *stream) {
  if (!ctx) return fail(ADHA_ERR_INVALID, "ctx is NULL");
  ADHA_TRY(validate_remap(src_l, src, src_cap, dst_l, dst, dst_cap));
  DeviceGuard g(ctx->c.device);
  return remap_one(&ctx->c, src_l, src, dst_l, dst, (hipStream_t)stream);
}

adha_status adha_remap_in_place(adha_ctx *ctx, const adha_layout *src_l, const adha_layout *dst_l, void *buf,
                                uint64_t buf_cap, void *stream) {
  if (!ctx || !src_l || !dst_l) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!src_l->d.shape.same(dst_l->d.shape)) return fail(ADHA_ERR_INVALID, "layouts describe different structs");
  const uint64_t need = std::max(src_l->d.nbytes, dst_l->d.nbytes);
  ADHA_TRY(check_dev_buf("buf", buf, buf_cap, need));
  LayoutDesc a, b;
  bool moves = false;
  ADHA_TRY(in_place_parts(src_l->d, dst_l->d, &a, &b, &moves));  // checks the regions on the host
  DeviceGuard g(ctx->c.device);
  return remap_in_place(&ctx->c, src_l->d, dst_l->d, buf, (hipStream_t)stream);
}

adha_status adha_remap_set_shape(adha_ctx *ctx, const adha_layout *src_l, const adha_layout *dst_l,
                                 const adha_tile_shape *shape) {
  if (!ctx || !src_l || !dst_l || !shape) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!src_l->d.shape.same(dst_l->d.shape)) return fail(ADHA_ERR_INVALID, "layouts describe different structs");
  TileShape d;
  ADHA_TRY(choose_shape(&ctx->c, src_l->d, dst_l->d, &d));
  TileShape s;
  s.R = shape->tile_records ? shape->tile_records : d.R;
  s.K = shape->slots ? shape->slots : d.K;
  s.shift = shape->pad_shift ? shape->pad_shift : d.shift;
  s.wg_per_cu = shape->wg_per_cu ? shape->wg_per_cu : d.wg_per_cu;
  if (shape->order > 2 || shape->nontemporal > 2) return fail(ADHA_ERR_INVALID, "order / nontemporal not in {0, 1, 2}");
  s.strided = shape->order ? shape->order - 1 : d.strided;
  s.nt = shape->nontemporal ? shape->nontemporal - 1 : d.nt;
  if (s.R != 0) {
    ADHA_TRY(check_shape(src_l->d, dst_l->d, s));
  }
  ctx->c.forced_shapes[{src_l->id, dst_l->id}] = s;
  return ADHA_OK;
}

adha_status adha_remap_get_shape(adha_ctx *ctx, const adha_layout *src_l, const adha_layout *dst_l,
                                 adha_tile_shape *out) {
  if (!ctx || !src_l || !dst_l || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  TileShape s;
  ADHA_TRY(shape_for(&ctx->c, src_l, dst_l, &s));
  out->tile_records = s.R;
  out->slots = s.K;
  out->pad_shift = s.shift;
  out->wg_per_cu = s.wg_per_cu;
  out->order = s.strided + 1;
  out->nontemporal = s.nt + 1;
  return ADHA_OK;
}

adha_status adha_remap_describe(const adha_layout *src_l, const adha_layout *dst_l, int32_t cu_count,
                                adha_remap_info *out) {
  if (!src_l || !dst_l || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!src_l->d.shape.same(dst_l->d.shape)) return fail(ADHA_ERR_INVALID, "layouts describe different structs");
  if (cu_count <= 0 || cu_count > 4096) return fail(ADHA_ERR_INVALID, "cu_count %d not in [1, 4096]", cu_count);
  Ctx tmp;
  tmp.cu_count = cu_count;
  TileShape s;
  ADHA_TRY(choose_shape(&tmp, src_l->d, dst_l->d, &s));
  RemapPrepared p;
  ADHA_TRY(remap_prepare(&tmp, {&src_l->d}, {nullptr}, {&dst_l->d}, {nullptr}, {s}, &p, false));
  out->shape.tile_records = s.R;
  out->shape.slots = s.K;
  out->shape.pad_shift = s.shift;
  out->shape.wg_per_cu = s.wg_per_cu;
  out->shape.order = s.strided + 1;
  out->shape.nontemporal = s.nt + 1;
  out->full_tiles = p.main_tiles;
  out->tail_bytes = p.tail_bytes;
  out->descriptor_bytes = p.desc_bytes;
  out->grid = p.grid;
  out->lds_bytes = p.lds;
  out->byte_path = p.byte_path;
  return ADHA_OK;
}

adha_status adha_remap_batched(adha_ctx *ctx, uint32_t n, const adha_remap_item *items, uint32_t flags,
                               void *stream) {
  if (!ctx) return fail(ADHA_ERR_INVALID, "ctx is NULL");
  if (n == 0) return ADHA_OK;
  if (!items) return fail(ADHA_ERR_INVALID, "items is NULL");
  for (uint32_t i = 0; i < n; ++i) {
    const adha_remap_item &it = items[i];
    adha_status st = validate_remap(it.src_layout, it.src, it.src_cap, it.dst_layout, it.dst, it.dst_cap);
    if (st < 0) return fail(st, "item %u: %s", i, adha::last_error());
  }
  ADHA_TRY(check_items_disjoint(n, items));
  DeviceGuard g(ctx->c.device);
  return batch_run(&ctx->c, n, items, flags, (hipStream_t)stream);
}

}  // extern "C"

// Batched remap of validated items under the context's batch policy.
adha_status adha::batch_run(Ctx *c, uint32_t n, const adha_remap_item *items, uint32_t flags, hipStream_t st) {
  if (flags & ADHA_BATCH_SEPARATE) {
    for (uint32_t i = 0; i < n; ++i)
      ADHA_TRY(remap_one(c, items[i].src_layout, items[i].src, items[i].dst_layout, items[i].dst, st));
    return ADHA_OK;
  }
  std::vector<const LayoutDesc *> sl, dl;
  std::vector<const void *> sp;
  std::vector<void *> dp;
  std::vector<TileShape> shapes;
  std::vector<uint64_t> key{2};
  for (uint32_t i = 0; i < n; ++i) {
    const adha_remap_item &it = items[i];
    if (it.src_layout->d.shape.n == 0 || it.dst_layout->d.nbytes == 0) continue;
    TileShape sh;
    ADHA_TRY(batch_shape_for(c, it.src_layout, it.dst_layout, &sh));
    sl.push_back(&it.src_layout->d);
    dl.push_back(&it.dst_layout->d);
    sp.push_back(it.src);
    dp.push_back(it.dst);
    shapes.push_back(sh);
    for (uint64_t v : {it.src_layout->id, it.dst_layout->id, (uint64_t)(uintptr_t)it.src,
                       (uint64_t)(uintptr_t)it.dst, (uint64_t)sh.R, (uint64_t)sh.K,
                       (uint64_t)sh.shift, (uint64_t)sh.wg_per_cu, (uint64_t)sh.strided, (uint64_t)sh.nt})
      key.push_back(v);
  }
  if (sl.empty()) return ADHA_OK;
  // a batch mixes arrays with different shifts only through its first entry
  for (auto &s : shapes) {
    s.shift = shapes[0].shift;
    s.strided = shapes[0].strided;
    s.nt = shapes[0].nt;
  }
  auto it = c->remap_cache.find(key);
  if (it == c->remap_cache.end()) {
    if (c->remap_cache.size() >= kCacheLimit) ADHA_TRY(flush_cache(c));
    RemapPrepared p;
    ADHA_TRY(remap_prepare(c, sl, sp, dl, dp, shapes, &p));
    it = c->remap_cache.emplace(key, p).first;
  }
  const RemapPrepared &P = it->second;
  if (!(flags & ADHA_BATCH_GRAPH)) return remap_run(c, P, nullptr, nullptr, st);

  GraphEntry *ge = nullptr;
  for (auto &e : c->graphs)
    if (e.key == key) ge = &e;
  if (!ge) {
    hipStream_t cap = nullptr;
    ADHA_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    GraphEntry e;
    e.key = key;
    hipError_t he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    adha_status rs = he == hipSuccess ? remap_run(c, P, nullptr, nullptr, cap) : ADHA_ERR_DEVICE;
    hipError_t he2 = hipStreamEndCapture(cap, &e.graph);
    (void)hipStreamDestroy(cap);
    if (he != hipSuccess || rs < 0 || he2 != hipSuccess) {
      if (e.graph) (void)hipGraphDestroy(e.graph);
      return fail(ADHA_ERR_DEVICE, "graph capture of the batched remap failed");
    }
    he = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
    if (he != hipSuccess) {
      (void)hipGraphDestroy(e.graph);
      return fail(ADHA_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(he));
    }
    c->graphs.push_back(e);
    ge = &c->graphs.back();
  }
  ADHA_HIP(hipGraphLaunch(ge->exec, st));
  return ADHA_OK;
}

extern "C" {

// ------------------------------------------------------------------ sections
adha_status adha_section_create(const adha_struct *s, adha_op op, uint32_t n_read, const int32_t *read,
                                uint32_t n_write, const int32_t *write, uint32_t degree,
                                adha_section **out) {
  if (!s || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  const Shape &sh = s->shape;
  const int F = sh.nfields();
  if (n_read == 0 || n_read > ADHA_MAX_READ)
    return fail(ADHA_ERR_INVALID, "n_read %u not in [1, %d]", n_read, ADHA_MAX_READ);
  if (n_write == 0 || n_write > ADHA_MAX_WRITE)
    return fail(ADHA_ERR_INVALID, "n_write %u not in [1, %d]", n_write, ADHA_MAX_WRITE);
  if (!read || !write) return fail(ADHA_ERR_INVALID, "read / write arrays are NULL");
  if (degree > ADHA_MAX_DEGREE) return fail(ADHA_ERR_INVALID, "degree %u > %d", degree, ADHA_MAX_DEGREE);
  SectionDesc d;
  d.shape = sh;
  d.op = enum_value(op);
  d.degree = degree;
  d.rd.assign(read, read + n_read);
  d.wr.assign(write, write + n_write);
  std::sort(d.rd.begin(), d.rd.end());
  std::sort(d.wr.begin(), d.wr.end());
  for (auto *v : {&d.rd, &d.wr}) {
    for (size_t i = 0; i < v->size(); ++i) {
      int f = (*v)[i];
      if (f < 0 || f >= F) return fail(ADHA_ERR_INVALID, "field id %d out of range", f);
      if (i && (*v)[i - 1] == f) return fail(ADHA_ERR_INVALID, "field id %d listed twice", f);
      if (sh.dtype[f] == ADHA_RAW) return fail(ADHA_ERR_UNSUPPORTED, "field %d is RAW; sections need typed fields", f);
    }
  }
  if (degree > 0) {
    for (int f : d.wr)
      if (std::find(d.rd.begin(), d.rd.end(), f) != d.rd.end())
        return fail(ADHA_ERR_INVALID, "gather section writes field %d that it reads (records would race)", f);
  }
  switch (enum_value(op)) {
    case ADHA_OP_GEN:
      break;
    case ADHA_OP_MULADD3:
    case ADHA_OP_SUB2:
    case ADHA_OP_SUM: {
      uint32_t need = op == ADHA_OP_MULADD3 ? 3 : op == ADHA_OP_SUB2 ? 2 : 0;
      if (need && n_read != need) return fail(ADHA_ERR_INVALID, "op needs exactly %u read fields", need);
      if (n_write != 1) return fail(ADHA_ERR_INVALID, "op writes exactly one field");
      if (degree) return fail(ADHA_ERR_UNSUPPORTED, "op is direct only");
      if (sh.dtype[d.wr[0]] != ADHA_F32 && sh.dtype[d.wr[0]] != ADHA_F64)
        return fail(ADHA_ERR_UNSUPPORTED, "op needs a floating-point write field");
      break;
    }
    case ADHA_OP_REDUCE:
      return fail(ADHA_ERR_INVALID, "reductions are created by adha_section_create_reduce");
    default:
      return fail(ADHA_ERR_INVALID, "unknown op %d", enum_value(op));
  }
  auto *sec = new (std::nothrow) adha_section;
  if (!sec) return fail(ADHA_ERR_OOM, "section allocation failed");
  sec->d = std::move(d);
  *out = sec;
  return ADHA_OK;
}

adha_status adha_section_create_stencil(const adha_struct *s, uint32_t n_read, const int32_t *read,
                                        uint32_t n_write, const int32_t *write, uint32_t nx, uint32_t ny,
                                        uint32_t nz, uint32_t d, const int32_t *offsets, adha_section **out) {
  if (!s || !out || !offsets) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (d == 0 || d > ADHA_MAX_DEGREE) return fail(ADHA_ERR_INVALID, "stencil degree %u not in [1, %d]", d, ADHA_MAX_DEGREE);
  if (s->shape.n >= (int64_t(1) << 31)) return fail(ADHA_ERR_UNSUPPORTED, "stencil grids hold fewer than 2^31 records");
  if ((uint64_t)nx * ny * nz != (uint64_t)s->shape.n || nx == 0 || ny == 0 || nz == 0)
    return fail(ADHA_ERR_INVALID, "grid %u x %u x %u does not hold the struct's %lld records", nx, ny, nz,
                (long long)s->shape.n);
  const uint32_t ext[3] = {nx, ny, nz};
  for (uint32_t j = 0; j < 3 * d; ++j)
    if ((uint64_t)std::abs((int64_t)offsets[j]) >= ext[j % 3])
      return fail(ADHA_ERR_INVALID, "offset %d of neighbour %u reaches past the grid", offsets[j], j / 3);
  adha_section *sec = nullptr;
  ADHA_TRY(adha_section_create(s, ADHA_OP_GEN, n_read, read, n_write, write, d, &sec));
  sec->d.stencil = true;
  sec->d.nx = nx;
  sec->d.ny = ny;
  sec->d.nz = nz;
  sec->d.offsets.assign(offsets, offsets + 3 * d);
  *out = sec;
  return ADHA_OK;
}

adha_status adha_section_create_reduce(const adha_struct *s, uint32_t n_read, const int32_t *read,
                                       int32_t key_field, uint32_t n_keys, void *out, uint64_t out_cap,
                                       adha_section **out_sec) {
  if (!s || !out_sec) return fail(ADHA_ERR_INVALID, "NULL argument");
  const Shape &sh = s->shape;
  const int F = sh.nfields();
  if (n_read == 0 || n_read > ADHA_MAX_READ)
    return fail(ADHA_ERR_INVALID, "n_read %u not in [1, %d]", n_read, ADHA_MAX_READ);
  if (!read) return fail(ADHA_ERR_INVALID, "read array is NULL");
  SectionDesc d;
  d.shape = sh;
  d.op = ADHA_OP_REDUCE;
  d.rd.assign(read, read + n_read);
  std::sort(d.rd.begin(), d.rd.end());
  for (size_t i = 0; i < d.rd.size(); ++i) {
    const int f = d.rd[i];
    if (f < 0 || f >= F) return fail(ADHA_ERR_INVALID, "field id %d out of range", f);
    if (i && d.rd[i - 1] == f) return fail(ADHA_ERR_INVALID, "field id %d listed twice", f);
    if (sh.dtype[f] == ADHA_RAW) return fail(ADHA_ERR_UNSUPPORTED, "field %d is RAW; sections need typed fields", f);
    if (sh.ebytes[f] < 4)
      return fail(ADHA_ERR_UNSUPPORTED, "field %d has %u-byte elements; reductions read 4- and 8-byte fields", f,
                  sh.ebytes[f]);
  }
  if (key_field >= 0) {
    if (key_field >= F) return fail(ADHA_ERR_INVALID, "key field %d out of range", key_field);
    if (sh.dtype[key_field] != ADHA_I32) return fail(ADHA_ERR_INVALID, "key field %d is not I32", key_field);
    if (std::find(d.rd.begin(), d.rd.end(), key_field) != d.rd.end())
      return fail(ADHA_ERR_INVALID, "key field %d is also read", key_field);
  } else if (key_field != -1) {
    return fail(ADHA_ERR_INVALID, "key field %d: use -1 for no key", key_field);
  } else if (n_keys != 1) {
    return fail(ADHA_ERR_INVALID, "a reduction without a key has one row, not %u", n_keys);
  }
  if (n_keys == 0) return fail(ADHA_ERR_INVALID, "n_keys is 0");
  if ((uint64_t)n_keys * (n_read + 1) > ADHA_MAX_REDUCE_CELLS)
    return fail(ADHA_ERR_INVALID, "table of %u x %u cells exceeds %d", n_keys, n_read + 1, ADHA_MAX_REDUCE_CELLS);
  d.key = key_field;
  d.n_keys = n_keys;
  const uint64_t need = (uint64_t)d.reduce_cells() * 8;
  ADHA_TRY(check_dev_buf("out", out, out_cap, need));
  d.out = out;
  d.out_cap = out_cap;
  auto *sec = new (std::nothrow) adha_section;
  if (!sec) return fail(ADHA_ERR_OOM, "section allocation failed");
  sec->d = std::move(d);
  *out_sec = sec;
  return ADHA_OK;
}

adha_status adha_section_destroy(adha_section *sec) {
  delete sec;
  return ADHA_OK;
}

adha_status adha_section_bytes(const adha_section *sec, uint64_t *out) {
  if (!sec || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  *out = sec->d.algorithmic_bytes();
  return ADHA_OK;
}

}  // extern "C"

namespace adha {
adha_status validate_section_run(const adha_section *sec, const adha_layout *l, const void *buf,
                                 uint64_t buf_cap, const int32_t *idx, uint64_t idx_count) {
  if (!sec || !l) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!sec->d.shape.same(l->d.shape)) return fail(ADHA_ERR_INVALID, "section and layout describe different structs");
  ADHA_TRY(check_dev_buf("buf", buf, buf_cap, l->d.nbytes));
  if (sec->d.degree > 0 && !sec->d.stencil && l->d.shape.n > 0) {
    if (!idx) return fail(ADHA_ERR_INVALID, "gather section needs an index array");
    if (!aligned(idx)) return fail(ADHA_ERR_INVALID, "idx is not 256-byte aligned");
    if (idx_count < (uint64_t)l->d.shape.n * sec->d.degree)
      return fail(ADHA_ERR_INVALID, "idx holds %llu entries, N*d = %llu are needed",
                  (unsigned long long)idx_count, (unsigned long long)l->d.shape.n * sec->d.degree);
    if (overlap(idx, idx_count * 4, buf, l->d.nbytes)) return fail(ADHA_ERR_INVALID, "idx overlaps buf");
  }
  if (sec->d.op == ADHA_OP_REDUCE && overlap(sec->d.out, (uint64_t)sec->d.reduce_cells() * 8, buf, l->d.nbytes))
    return fail(ADHA_ERR_INVALID, "the reduction's result table overlaps buf");
  return ADHA_OK;
}
}  // namespace adha

extern "C" {

adha_status adha_section_run(adha_ctx *ctx, const adha_section *sec, const adha_layout *l, void *buf,
                             uint64_t buf_cap, const int32_t *idx, uint64_t idx_count, void *stream) {
  if (!ctx) return fail(ADHA_ERR_INVALID, "ctx is NULL");
  ADHA_TRY(validate_section_run(sec, l, buf, buf_cap, idx, idx_count));
  DeviceGuard g(ctx->c.device);
  return section_launch(&ctx->c, sec->d, l->d, buf, idx, (hipStream_t)stream);
}

adha_status adha_section_run_static(adha_ctx *ctx, const adha_section *sec, const adha_layout *l, void *buf,
                                    uint64_t buf_cap, const int32_t *idx, uint64_t idx_count, void *stream) {
  if (!ctx) return fail(ADHA_ERR_INVALID, "ctx is NULL");
  ADHA_TRY(validate_section_run(sec, l, buf, buf_cap, idx, idx_count));
  if (!ctx->c.static_scratch) return fail(ADHA_ERR_STATE, "the context has no static scratch address");
  if (sec->d.op == ADHA_OP_REDUCE) {
    const ReducePlan p = reduce_plan(&ctx->c, sec->d, l->d.shape.n);
    if (p.partial_bytes > kReducePartialPairs * 16)
      return fail(ADHA_ERR_INVALID, "the reduction's partials need %llu bytes, more than the %llu of the static scratch",
                  (unsigned long long)p.partial_bytes, (unsigned long long)(kReducePartialPairs * 16));
  }
  DeviceGuard g(ctx->c.device);
  return section_launch(&ctx->c, sec->d, l->d, buf, idx, (hipStream_t)stream, nullptr, ctx->c.static_scratch);
}

}  // extern "C"
