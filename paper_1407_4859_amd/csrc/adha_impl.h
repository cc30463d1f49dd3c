// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "adha.h"

namespace adha {

// The integer a caller passed for an enum parameter or option field, read
// from its bytes: a value outside the enumerators (an invalid argument from
// C or Python) is then an ordinary int to reject, not a load of an enum
// outside its range.
template <class E>
inline int32_t enum_value(const E &e) {
  static_assert(sizeof(E) == sizeof(int32_t), "C-ABI enums are 32-bit");
  int32_t v;
  std::memcpy(&v, &e, sizeof v);
  return v;
}

// ------------------------------------------------------------------ errors
adha_status fail(adha_status st, const char *fmt, ...);
void clear_error();

#define ADHA_TRY(expr)                 \
  do {                                 \
    adha_status st_ = (expr);          \
    if (st_ < 0) return st_;           \
  } while (0)

#define ADHA_HIP(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::adha::fail(ADHA_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------ shapes
struct Shape {
  int64_t n = 0;
  std::vector<int32_t> dtype;
  std::vector<uint32_t> ebytes;
  int nfields() const { return (int)ebytes.size(); }
  uint32_t record_bytes() const {
    uint32_t s = 0;
    for (auto e : ebytes) s += e;
    return s;
  }
  bool same(const Shape &o) const { return n == o.n && dtype == o.dtype && ebytes == o.ebytes; }
};

struct Group {
  std::vector<int> fields;  // ascending
  uint32_t T = 1, logT = 0, S = 0;
  uint64_t base = 0, bytes = 0;  // bytes = roundup(N, T) * S
};

// Canonical layout: groups ordered by smallest field id, fields packed.
struct LayoutDesc {
  Shape shape;
  std::vector<Group> groups;
  std::vector<uint32_t> group_of, p;  // per field: group index, byte offset in group record
  uint64_t nbytes = 0;

  uint64_t addr(int64_t r, int f) const {
    const Group &g = groups[group_of[f]];
    return g.base + (uint64_t)(r >> g.logT) * g.T * g.S + (uint64_t)p[f] * g.T +
           (uint64_t)(r & (g.T - 1)) * shape.ebytes[f];
  }
  // end of the region group gi owns: its records, its padding records and
  // the padding up to the next multiple of 256 (in a canonical layout that
  // is where the next group starts)
  uint64_t group_end(size_t gi) const { return groups[gi].base + (groups[gi].bytes + 255) / 256 * 256; }
  bool placed = false;  // group bases given explicitly (adha_layout_place), not canonical
  // same shape, groups, tiles and group bases
  bool same_map(const LayoutDesc &o) const;
  // same shape, groups and tiles (bases may differ)
  bool same_groups(const LayoutDesc &o) const;
  bool dword_fields() const;   // every element is 4 or 8 bytes
  uint32_t max_tile() const;
  int layout_class() const;    // 0 AoS, 1 SoA, 2 tiled, 3 grouped interleaved / mixed
};

adha_status build_layout(const Shape &sh, uint32_t n_groups, const uint32_t *gof,
                         const uint32_t *tog, LayoutDesc *out);
LayoutDesc layout_aos(const Shape &sh, uint32_t tile = 1);
LayoutDesc layout_soa(const Shape &sh);
LayoutDesc layout_from_parts(const Shape &sh, const std::vector<std::vector<int>> &parts,
                             uint32_t tile);
// Gives the groups explicit bases (one per group, in group order, multiples
// of 256, regions [base, group_end) disjoint); nbytes becomes the last end.
adha_status place_layout(LayoutDesc *L, const std::vector<uint64_t> &bases);
// The two groups hold the same fields with the same tile.
inline bool same_group(const Group &a, const Group &b) { return a.T == b.T && a.fields == b.fields; }
// Fields whose group (fields and tile) differs between a and b: the fields
// a remap a -> b has to move when groups that agree stay where they are.
std::vector<int> moving_fields(const LayoutDesc &a, const LayoutDesc &b);
// Group placement for a sequence of layouts run one after another in one
// buffer: seq[0] at its canonical bases; for every later layout, a group
// that the previous one holds with the same fields and tile keeps its base,
// and every other group goes to the lowest 256-aligned offset clear of all
// of the previous layout's groups and of the new groups placed before it.
// out[i] is seq[i] placed; *arena the bytes the whole sequence needs.
void place_sequence(const std::vector<const LayoutDesc *> &seq, std::vector<LayoutDesc> *out, uint64_t *arena);
// The sub-remap that an in-place remap src -> dst performs: the fields that
// move, as a struct of their own, with the source groups they leave and the
// destination groups they enter (bases kept).  false when nothing moves.
// Fails when a destination group that moves overlaps a source group.
adha_status in_place_parts(const LayoutDesc &src, const LayoutDesc &dst, LayoutDesc *sub_src, LayoutDesc *sub_dst,
                           bool *moves);

struct SectionDesc {
  Shape shape;
  int32_t op = 0;
  std::vector<int32_t> rd, wr;
  uint32_t degree = 0;
  // stencils: neighbours at grid offsets instead of an index array
  bool stencil = false;
  uint32_t nx = 0, ny = 0, nz = 0;
  std::vector<int32_t> offsets;  // 3 per neighbour
  // reductions: key field (-1: none), key count, result table (device)
  int32_t key = -1;
  uint32_t n_keys = 1;
  void *out = nullptr;
  uint64_t out_cap = 0;
  uint64_t algorithmic_bytes() const;
  // every field read at the record itself in a direct pass: the read
  // fields plus a reduction's key
  std::vector<int32_t> streamed_reads() const {
    std::vector<int32_t> v = rd;
    if (key >= 0) {
      v.push_back(key);
      std::sort(v.begin(), v.end());
    }
    return v;
  }
  uint32_t reduce_cells() const { return n_keys * ((uint32_t)rd.size() + 1); }
};

}  // namespace adha

// --------------------------------------------------------------- handles
struct adha_struct {
  adha::Shape shape;
};
struct adha_layout {
  adha::LayoutDesc d;
  uint64_t id;
};
struct adha_section {
  adha::SectionDesc d;
};
struct adha_program {
  adha::Shape shape;
  std::vector<adha::SectionDesc> secs;
  // control flow: empty = the sections in order; otherwise section indices
  // and IF / ELSE / END markers, with one probability per IF
  std::vector<int32_t> tokens;
  std::vector<double> probs;
};

namespace adha {

uint64_t next_layout_id();
adha_layout *new_layout(LayoutDesc d);

// ------------------------------------------------------------------ remap
struct TileShape {
  uint32_t R = 0, K = 0, shift = 0, wg_per_cu = 0;
  uint32_t strided = 0, nt = 0;  // tile order across workgroups; streaming accesses
};

struct Ctx;
// A remap launch, prepared once: its descriptor blob lives in device memory
// (owned by the context's cache) and only kernel launches remain.
struct RemapPrepared {
  uint8_t *dev = nullptr;           // blob allocation
  const uint8_t *arrays = nullptr;  // every array (tail kernel)
  const uint8_t *main_arrays = nullptr;  // arrays with full tiles (main kernel)
  const uint8_t *tails = nullptr;
  uint64_t main_tiles = 0, tiles_per_wg = 0, grid = 0, tail_blocks = 0;
  uint32_t n_arrays = 0, n_main = 0, n_tails = 0;
  uint32_t K = 1, shift = 6, wg_per_cu = 1, lds = 0, strided = 0, nt = 0;
  uint32_t byte_path = 0;  // some array has 1- or 2-byte fields: main kernel in byte mode
  uint64_t desc_bytes = 0, tail_bytes = 0;
};
// Builds the descriptor blob of a launch; with upload it is copied into a
// new device allocation (owned by the caller through RemapPrepared::dev).
adha_status remap_prepare(Ctx *ctx, const std::vector<const LayoutDesc *> &src_l,
                          const std::vector<const void *> &src,
                          const std::vector<const LayoutDesc *> &dst_l,
                          const std::vector<void *> &dst, const std::vector<TileShape> &shapes,
                          RemapPrepared *out, bool upload = true);
// src_override / dst_override replace the (single) array's pointers when set.
adha_status remap_run(Ctx *ctx, const RemapPrepared &p, const void *src_override,
                      void *dst_override, hipStream_t stream);
adha_status choose_shape(const Ctx *ctx, const LayoutDesc &a, const LayoutDesc &b, TileShape *out);
// Shape from a policy: the largest multiple of max(64, T) records within
// tile_bytes (at least one such multiple), slots to match.
adha_status policy_shape(const LayoutDesc &a, const LayoutDesc &b, uint32_t tile_bytes, uint32_t wg_per_cu,
                         uint32_t strided, uint32_t nt, TileShape *out);
std::string tune_key(const LayoutDesc &a, const LayoutDesc &b);
uint32_t default_tile_bytes(const LayoutDesc &a);
adha_status check_shape(const LayoutDesc &a, const LayoutDesc &b, const TileShape &s);
uint32_t remap_lds_bytes(const LayoutDesc &a, const TileShape &s);

adha_status validate_remap(const adha_layout *sl, const void *src, uint64_t src_cap, const adha_layout *dl,
                           const void *dst, uint64_t dst_cap);
adha_status shape_for(Ctx *ctx, const adha_layout *a, const adha_layout *b, TileShape *sh);
adha_status remap_with_shape(Ctx *ctx, const adha_layout *sl, const void *src, const adha_layout *dl,
                             void *dst, const TileShape &sh, hipStream_t stream);
adha_status batch_run(Ctx *c, uint32_t n, const adha_remap_item *items, uint32_t flags, hipStream_t st);
// In one buffer: writes the groups of dst that src does not hold at the same
// base (same fields and tile), from where src holds their fields.
adha_status remap_in_place(Ctx *ctx, const LayoutDesc &src, const LayoutDesc &dst, void *buf, hipStream_t stream);
// No item's destination overlaps another item's destination or source.
adha_status check_items_disjoint(uint32_t n, const adha_remap_item *items);
adha_status prepared_for(Ctx *ctx, const adha_layout *a, const adha_layout *b, const TileShape &sh,
                         const RemapPrepared **out);

// ------------------------------------------------------------------ sections
// scratch: device memory for a reduction's per-workgroup partials (at least
// kReducePartialPairs * 16 bytes); NULL = the context's own.
adha_status section_launch(Ctx *ctx, const SectionDesc &sec, const LayoutDesc &l, void *buf,
                           const int32_t *idx, hipStream_t stream, void *out_override = nullptr,
                           void *scratch = nullptr);

// Reductions: pass 1 writes one partial table of (double, double) pairs per
// workgroup; workgroups x cells never exceeds this many pairs (16 MiB).
static const uint64_t kReducePartialPairs = 1ull << 20;
struct ReducePlan {
  uint32_t keys_in_regs = 0;  // 1..8: register form with that many key rows; 0: LDS form
  uint32_t slot_cols = 0;     // > 0: slot form (F32 reads, 3..8 keys) with this slice width
  uint32_t slices = 1;        // column slices (gridDim.y) of the register form
  uint32_t groups = 1;        // workgroups per slice
  size_t lds = 0;             // dynamic LDS of the LDS and slot forms
  uint64_t partial_bytes = 0;
};
ReducePlan reduce_plan(const Ctx *ctx, const SectionDesc &sec, int64_t n);
adha_status reduce_launch(Ctx *ctx, const SectionDesc &sec, const LayoutDesc &l, const void *buf, void *out,
                          uint64_t *partials, uint64_t partial_cap, hipStream_t stream);

// ------------------------------------------------------------------ host backend
uint32_t host_threads(const Ctx *ctx);
// A section on host memory; a reduction writes its table (host) to `table`.
// *bad_out counts out-of-range gather indices or reduction keys.
adha_status host_section_run(uint32_t threads, const SectionDesc &sec, const LayoutDesc &l, uint8_t *buf,
                             const int32_t *idx, void *table, uint64_t *bad_out);
adha_status host_remap(uint32_t threads, const LayoutDesc &a, const uint8_t *src, const LayoutDesc &b,
                       uint8_t *dst);

// ------------------------------------------------------------------ MLP
// At most this many networks in a cost model (their mean prediction is used).
static const uint32_t kMaxEnsemble = 16;
adha_status mlp_forward(Ctx *ctx, const float *params, const float *x, uint32_t batch, float *y,
                        hipStream_t stream);
// scratch holds scratch_floats floats; the call fails (before any launch)
// when the batch needs more than that (mlp_scratch_floats(batch)).
adha_status mlp_backward(Ctx *ctx, const float *params, const float *x, const float *target,
                         uint32_t batch, float *grad, float *loss, float *scratch,
                         size_t scratch_floats, hipStream_t stream);
adha_status mlp_adam(Ctx *ctx, float *params, const float *grad, float *m, float *v, float lr,
                     float b1, float b2, float eps, uint32_t t, hipStream_t stream);
size_t mlp_scratch_floats(uint32_t batch);

// ------------------------------------------------------------------ context
struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct Ctx {
  int device = 0;
  std::map<std::vector<uint64_t>, RemapPrepared> remap_cache;
  int cu_count = 256;
  std::string arch;
  uint32_t *err_flag = nullptr;  // device word: gather index out of range seen
  std::map<std::tuple<uint64_t, uint64_t>, TileShape> forced_shapes;
  std::map<std::string, TileShape> tunedb;  // tuned shapes by layout-pair class
  struct BatchPolicy {
    uint32_t tile_bytes = 16384, wg_per_cu = 4, strided = 0, nt = 1;
  } batch;
  std::vector<GraphEntry> graphs;
  std::vector<float> model;  // trained / loaded cost-model parameters, n_models networks (empty = none)
  uint32_t n_models = 1;
  bool has_model = false;
  // cost-model inference: parameters on the device (stale when !mlp_params_ok)
  // and grow-only feature / prediction buffers of mlp_io_cap rows
  float *mlp_params = nullptr, *mlp_x = nullptr, *mlp_y = nullptr;
  bool mlp_params_ok = false;
  uint32_t mlp_io_cap = 0;
  bool no_span = false;      // gathers always take the per-field path
  uint32_t reduce_wg_per_cu = 8;     // reductions: first-pass workgroups per CU
  bool reduce_plain = false;         // reductions: plain double sums instead of compensated ones
  void *reduce_partials = nullptr;   // reductions: kReducePartialPairs * 16 bytes, allocated on first use
  void *static_scratch = nullptr;    // the device address of this device's static scratch array
  uint32_t host_threads = 0;         // host backend threads (0: one per core, at most 64)
  uint64_t host_bad = 0;             // out-of-range indices / keys met by host sections
  ~Ctx();
};

// Allocates the context's reduction partials once (no-op when present).
adha_status ctx_reduce_scratch(Ctx *ctx);
// Device address of `device`'s static scratch array (kReducePartialPairs * 16
// bytes), looked up once per device with that device current.
adha_status static_scratch_address(int device, void **out);

// Switches to the context's device for the lifetime of the guard.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

}  // namespace adha

struct adha_ctx {
  adha::Ctx c;
};
