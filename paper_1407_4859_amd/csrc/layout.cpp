// Layout descriptors: canonicalisation and the address map.
//
// The paper's layouts (AoS, SoA, and structures of clustered fields such as
// Table 2's AoSU / AoSV and Table 3's four 8-field structures) are all
// partitions of the fields into groups; a group is interleaved (tile 1) or
// stored as tiles of T records (AoSoA).
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>

#include "adha_impl.h"

namespace adha {

static thread_local std::string g_err;

adha_status fail(adha_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

void clear_error() { g_err.clear(); }

const char *last_error() { return g_err.c_str(); }

static uint64_t roundup(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

static std::atomic<uint64_t> g_layout_ids{1};
uint64_t next_layout_id() { return g_layout_ids.fetch_add(1); }

adha_layout *new_layout(LayoutDesc d) {
  auto *l = new (std::nothrow) adha_layout;
  if (!l) return nullptr;
  l->d = std::move(d);
  l->id = next_layout_id();
  return l;
}

static void finish(LayoutDesc &L) {
  const Shape &sh = L.shape;
  std::sort(L.groups.begin(), L.groups.end(),
            [](const Group &a, const Group &b) { return a.fields[0] < b.fields[0]; });
  L.group_of.assign(sh.nfields(), 0);
  L.p.assign(sh.nfields(), 0);
  uint64_t at = 0;
  for (size_t gi = 0; gi < L.groups.size(); ++gi) {
    Group &g = L.groups[gi];
    std::sort(g.fields.begin(), g.fields.end());
    if (g.fields.size() == 1) g.T = 1;
    g.logT = 0;
    while ((1u << g.logT) < g.T) ++g.logT;
    uint32_t s = 0;
    for (int f : g.fields) {
      L.group_of[f] = (uint32_t)gi;
      L.p[f] = s;
      s += sh.ebytes[f];
    }
    g.S = s;
    g.bytes = roundup((uint64_t)sh.n, g.T) * s;
    g.base = at;
    at = roundup(at + g.bytes, 256);
  }
  L.nbytes = at;
}

adha_status build_layout(const Shape &sh, uint32_t n_groups, const uint32_t *gof,
                         const uint32_t *tog, LayoutDesc *out) {
  const int F = sh.nfields();
  if (F == 0) return fail(ADHA_ERR_INVALID, "struct has no fields");
  if (!gof || !tog) return fail(ADHA_ERR_INVALID, "group_of_field and tile_of_group are required");
  if (n_groups == 0 || n_groups > (uint32_t)F)
    return fail(ADHA_ERR_INVALID, "n_groups %u not in [1, %d]", n_groups, F);
  LayoutDesc L;
  L.shape = sh;
  L.groups.resize(n_groups);
  for (int f = 0; f < F; ++f) {
    if (gof[f] >= n_groups)
      return fail(ADHA_ERR_INVALID, "field %d has group label %u >= n_groups %u", f, gof[f], n_groups);
    L.groups[gof[f]].fields.push_back(f);
  }
  for (uint32_t g = 0; g < n_groups; ++g) {
    if (L.groups[g].fields.empty()) return fail(ADHA_ERR_INVALID, "group label %u has no field", g);
    uint32_t t = tog[g];
    if (t == 0 || t > ADHA_MAX_TILE || (t & (t - 1)))
      return fail(ADHA_ERR_INVALID, "tile %u of group %u is not a power of two in [1, %d]", t, g,
                  ADHA_MAX_TILE);
    L.groups[g].T = t;
  }
  finish(L);
  *out = std::move(L);
  return ADHA_OK;
}

LayoutDesc layout_aos(const Shape &sh, uint32_t tile) {
  LayoutDesc L;
  L.shape = sh;
  Group g;
  for (int f = 0; f < sh.nfields(); ++f) g.fields.push_back(f);
  g.T = tile;
  L.groups.push_back(g);
  finish(L);
  return L;
}

LayoutDesc layout_soa(const Shape &sh) {
  LayoutDesc L;
  L.shape = sh;
  for (int f = 0; f < sh.nfields(); ++f) {
    Group g;
    g.fields.push_back(f);
    L.groups.push_back(g);
  }
  finish(L);
  return L;
}

LayoutDesc layout_from_parts(const Shape &sh, const std::vector<std::vector<int>> &parts,
                             uint32_t tile) {
  LayoutDesc L;
  L.shape = sh;
  std::vector<char> used(sh.nfields(), 0);
  for (auto &p : parts) {
    Group g;
    g.fields = p;
    g.T = tile;
    for (int f : p) used[f] = 1;
    L.groups.push_back(g);
  }
  for (int f = 0; f < sh.nfields(); ++f)
    if (!used[f]) {
      Group g;
      g.fields.push_back(f);
      L.groups.push_back(g);
    }
  finish(L);
  return L;
}

bool LayoutDesc::same_groups(const LayoutDesc &o) const {
  if (!shape.same(o.shape) || groups.size() != o.groups.size()) return false;
  for (size_t i = 0; i < groups.size(); ++i)
    if (!same_group(groups[i], o.groups[i])) return false;
  return true;
}

bool LayoutDesc::same_map(const LayoutDesc &o) const {
  if (!same_groups(o)) return false;
  for (size_t i = 0; i < groups.size(); ++i)
    if (groups[i].base != o.groups[i].base) return false;
  return true;
}

adha_status place_layout(LayoutDesc *L, const std::vector<uint64_t> &bases) {
  if (bases.size() != L->groups.size())
    return fail(ADHA_ERR_INVALID, "%zu bases given for %zu groups", bases.size(), L->groups.size());
  std::vector<std::pair<uint64_t, uint64_t>> spans;
  for (size_t g = 0; g < bases.size(); ++g) {
    if (bases[g] & 255u) return fail(ADHA_ERR_INVALID, "base %llu of group %zu is not a multiple of 256",
                                     (unsigned long long)bases[g], g);
    if (bases[g] > (1ull << 50)) return fail(ADHA_ERR_INVALID, "base of group %zu is too large", g);
    const uint64_t size = (L->groups[g].bytes + 255) / 256 * 256;
    if (size) spans.push_back({bases[g], bases[g] + size});
  }
  std::sort(spans.begin(), spans.end());
  for (size_t i = 1; i < spans.size(); ++i)
    if (spans[i].first < spans[i - 1].second) return fail(ADHA_ERR_INVALID, "group regions overlap");
  uint64_t end = 0;
  for (size_t g = 0; g < bases.size(); ++g) {
    L->groups[g].base = bases[g];
    end = std::max(end, L->group_end(g));
  }
  L->nbytes = end;
  L->placed = true;
  return ADHA_OK;
}

std::vector<int> moving_fields(const LayoutDesc &a, const LayoutDesc &b) {
  std::vector<int> out;
  for (int f = 0; f < a.shape.nfields(); ++f)
    if (!same_group(a.groups[a.group_of[f]], b.groups[b.group_of[f]])) out.push_back(f);
  return out;
}

void place_sequence(const std::vector<const LayoutDesc *> &seq, std::vector<LayoutDesc> *out, uint64_t *arena) {
  out->clear();
  *arena = 0;
  if (seq.empty()) return;
  out->push_back(*seq[0]);
  *arena = seq[0]->nbytes;
  for (size_t i = 1; i < seq.size(); ++i) {
    const LayoutDesc &prev = out->back();
    LayoutDesc L = *seq[i];
    std::vector<uint64_t> bases(L.groups.size(), 0);
    std::vector<std::pair<uint64_t, uint64_t>> busy;  // regions that may not be written
    for (size_t h = 0; h < prev.groups.size(); ++h)
      if (prev.groups[h].bytes) busy.push_back({prev.groups[h].base, prev.group_end(h)});
    std::vector<char> stays(L.groups.size(), 0);
    for (size_t g = 0; g < L.groups.size(); ++g)
      for (size_t h = 0; h < prev.groups.size(); ++h)
        if (same_group(L.groups[g], prev.groups[h])) {
          bases[g] = prev.groups[h].base;
          stays[g] = 1;
        }
    for (size_t g = 0; g < L.groups.size(); ++g) {
      if (stays[g]) continue;
      const uint64_t size = (L.groups[g].bytes + 255) / 256 * 256;
      std::sort(busy.begin(), busy.end());
      uint64_t at = 0;
      for (auto &sp : busy) {
        if (at + size <= sp.first) break;
        at = std::max(at, sp.second);
      }
      bases[g] = at;
      if (size) busy.push_back({at, at + size});
    }
    (void)place_layout(&L, bases);  // disjoint by construction
    *arena = std::max(*arena, L.nbytes);
    out->push_back(std::move(L));
  }
}

adha_status in_place_parts(const LayoutDesc &src, const LayoutDesc &dst, LayoutDesc *sub_src, LayoutDesc *sub_dst,
                           bool *moves) {
  if (!src.shape.same(dst.shape)) return fail(ADHA_ERR_INVALID, "the layouts describe different structs");
  const int F = src.shape.nfields();
  // a destination group stays when the source holds it at the same base
  std::vector<char> stay_d(dst.groups.size(), 0), stay_s(src.groups.size(), 0);
  for (size_t g = 0; g < dst.groups.size(); ++g)
    for (size_t h = 0; h < src.groups.size(); ++h)
      if (same_group(dst.groups[g], src.groups[h]) && dst.groups[g].base == src.groups[h].base) {
        stay_d[g] = 1;
        stay_s[h] = 1;
      }
  std::vector<int> newid(F, -1);
  Shape sub;
  sub.n = src.shape.n;
  for (int f = 0; f < F; ++f)
    if (!stay_d[dst.group_of[f]]) {
      newid[f] = sub.nfields();
      sub.dtype.push_back(src.shape.dtype[f]);
      sub.ebytes.push_back(src.shape.ebytes[f]);
    }
  *moves = sub.nfields() > 0;
  if (!*moves) return ADHA_OK;
  // a moving destination group may not overlap a source group that moves
  for (size_t g = 0; g < dst.groups.size(); ++g) {
    if (stay_d[g] || !dst.groups[g].bytes) continue;
    const uint64_t a = dst.groups[g].base, b = dst.group_end(g);
    for (size_t h = 0; h < src.groups.size(); ++h) {
      if (stay_s[h] || !src.groups[h].bytes) continue;
      const uint64_t c = src.groups[h].base, d = src.group_end(h);
      if (a < d && c < b) return fail(ADHA_ERR_INVALID, "destination group %zu overlaps source group %zu", g, h);
    }
  }
  auto part = [&](const LayoutDesc &L, const std::vector<char> &stay, LayoutDesc *out) {
    LayoutDesc P;
    P.shape = sub;
    std::vector<uint64_t> bases;
    for (size_t g = 0; g < L.groups.size(); ++g) {
      if (stay[g]) continue;
      Group G = L.groups[g];
      for (int &f : G.fields) f = newid[f];
      bases.push_back(G.base);
      P.groups.push_back(G);
    }
    // the fields keep their relative order, so the canonical finish gives
    // the same group order, offsets and sizes; then the real bases
    finish(P);
    std::vector<uint64_t> ordered(P.groups.size());
    for (size_t g = 0; g < P.groups.size(); ++g) ordered[g] = bases[g];
    return place_layout(&P, ordered) >= 0 ? (*out = std::move(P), true) : false;
  };
  if (!part(src, stay_s, sub_src) || !part(dst, stay_d, sub_dst))
    return fail(ADHA_ERR_INVALID, "inconsistent group placement");
  return ADHA_OK;
}

bool LayoutDesc::dword_fields() const {
  for (auto e : shape.ebytes)
    if (e != 4 && e != 8) return false;
  return true;
}

uint32_t LayoutDesc::max_tile() const {
  uint32_t t = 1;
  for (auto &g : groups) t = std::max(t, g.T);
  return t;
}

int LayoutDesc::layout_class() const {
  if (groups.size() == 1) return groups[0].T == 1 ? 0 : 2;
  bool all_single = true, any_tiled = false;
  for (auto &g : groups) {
    if (g.fields.size() > 1) all_single = false;
    if (g.T > 1) any_tiled = true;
  }
  if (all_single) return 1;
  return any_tiled ? 2 : 3;
}

uint64_t SectionDesc::algorithmic_bytes() const {
  uint64_t rb = 0, wb = 0;
  for (int f : rd) rb += shape.ebytes[f];
  for (int f : wr) wb += shape.ebytes[f];
  uint64_t n = (uint64_t)shape.n;
  if (key >= 0) rb += shape.ebytes[key];
  // a stencil's neighbours are records of the same arrays: at the minimum
  // every element is read once, as in a direct pass
  if (degree == 0 || stencil) return n * (rb + wb);
  return n * (4ull * degree + (uint64_t)degree * rb + wb);
}

}  // namespace adha
