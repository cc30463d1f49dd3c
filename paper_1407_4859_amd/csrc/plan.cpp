// Two-level layout selection and plan execution.
//
// Level 1, the ODS pass (section 2): an affinity graph over the fields a
// run of sections touches, then greedy clustering of the fields into
// structures no larger than a capacity in bytes.
// Level 2, the PDL pass (section 2): the sections in program order form a
// layered DAG whose nodes are (section, candidate layout); keeping a layout
// between consecutive sections is the paper's "combine" choice (the layout
// of a combined run is the ODS of the merged sections), changing it costs a
// "remap"; a shortest path gives the program layout.  Edge weights come from
// a profile of section times (measured on the device, the analytic bytes
// model, or the learned model).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <new>

#include "adha_impl.h"

struct adha_plan {
  adha::Shape shape;
  std::vector<adha::SectionDesc> secs;
  std::vector<adha_layout *> cands;
  std::vector<uint32_t> choice;  // per section: candidate layout
  std::vector<int32_t> dev;      // per section: 0 the GPU, 1 the host
  std::vector<double> T, R;  // k*C and C*C, microseconds (the GPU)
  // plans over both devices: host section costs (k*C), the host remap, the
  // transfers each way; a move between devices that changes the layout
  // remaps on the GPU side
  bool hetero = false;
  std::vector<double> TH;
  double rem_h = 0.0, xfer_dh = 0.0, xfer_hd = 0.0;
  // structured programs: the control flow and the candidate at each join
  // (kNoJoin: keep whatever layout the branch ends in)
  std::vector<int32_t> tokens;
  std::vector<double> probs;
  std::vector<uint32_t> join;
  double cost = 0.0, seconds = 0.0;
  // placed execution in one arena (adha_run_placed): the layout the data
  // starts in, then section s's layout at s + 1, with the groups two
  // consecutive layouts share kept in place; empty for structured programs
  // and plans over both devices.  `whole`: the remap costs are those of
  // whole-struct remaps (the executors that remap between two buffers).
  std::vector<adha_layout *> placed;
  uint64_t arena = 0;
  bool whole = false;
  uint32_t verified = 0;  // learned plans: (section, candidate) entries timed to verify the path
  ~adha_plan() {
    for (auto *l : cands) delete l;
    for (auto *l : placed) delete l;
  }
};

namespace adha {

adha_status remap_one(Ctx *ctx, const adha_layout *sl, const void *src, const adha_layout *dl,
                      void *dst, hipStream_t stream);
adha_status validate_section_run(const adha_section *sec, const adha_layout *l, const void *buf,
                                 uint64_t buf_cap, const int32_t *idx, uint64_t idx_count);
adha_status fill_uniform_index(int32_t *idx, uint64_t count, int64_t n, uint64_t seed, hipStream_t stream);
adha_status predict_costs(Ctx *ctx, const std::vector<std::vector<float>> &feats, const std::vector<double> &base_us,
                          std::vector<double> *us, hipStream_t stream);
void section_features(const SectionDesc &s, const LayoutDesc &l, float *out);

// ------------------------------------------------------------------ affinity
std::vector<uint64_t> affinity(const std::vector<SectionDesc> &secs, size_t first, size_t last, int F) {
  std::vector<uint64_t> w((size_t)F * F, 0);
  auto bump = [&](const std::vector<int32_t> &ids, uint64_t amount) {
    for (size_t x = 0; x < ids.size(); ++x)
      for (size_t y = x + 1; y < ids.size(); ++y) {
        w[(size_t)ids[x] * F + ids[y]] += amount;
        w[(size_t)ids[y] * F + ids[x]] += amount;
      }
  };
  for (size_t s = first; s <= last; ++s) {
    const SectionDesc &d = secs[s];
    if (d.degree == 0) {
      std::vector<int32_t> all = d.streamed_reads();
      for (int f : d.wr)
        if (std::find(all.begin(), all.end(), f) == all.end()) all.push_back(f);
      std::sort(all.begin(), all.end());
      bump(all, 1);
    } else {
      bump(d.rd, d.degree);
      bump(d.wr, 1);
    }
  }
  return w;
}

// Greedy clustering: edges by decreasing weight (ties by smaller then larger
// id); an edge joins its two clusters when they differ and fit the cap.
std::vector<std::vector<int>> ods_parts(const std::vector<SectionDesc> &secs, size_t first, size_t last,
                                        const Shape &sh, uint32_t cap) {
  const int F = sh.nfields();
  auto w = affinity(secs, first, last, F);
  struct E {
    uint64_t w;
    int a, b;
  };
  std::vector<E> edges;
  for (int a = 0; a < F; ++a)
    for (int b = a + 1; b < F; ++b)
      if (w[(size_t)a * F + b] > 0) edges.push_back({w[(size_t)a * F + b], a, b});
  std::sort(edges.begin(), edges.end(), [](const E &x, const E &y) {
    if (x.w != y.w) return x.w > y.w;
    if (x.a != y.a) return x.a < y.a;
    return x.b < y.b;
  });
  std::vector<int> cl(F);
  std::vector<uint64_t> bytes(F);
  for (int f = 0; f < F; ++f) {
    cl[f] = f;
    bytes[f] = sh.ebytes[f];
  }
  for (const E &e : edges) {
    int ca = cl[e.a], cb = cl[e.b];
    if (ca == cb || bytes[ca] + bytes[cb] > cap) continue;
    int keep = std::min(ca, cb), drop = std::max(ca, cb);
    for (int f = 0; f < F; ++f)
      if (cl[f] == drop) cl[f] = keep;
    bytes[keep] += bytes[drop];
  }
  std::vector<std::vector<int>> parts;
  for (int c = 0; c < F; ++c) {
    std::vector<int> m;
    for (int f = 0; f < F; ++f)
      if (cl[f] == c) m.push_back(f);
    if (m.size() > 1) parts.push_back(m);
  }
  std::sort(parts.begin(), parts.end());
  return parts;
}

// ------------------------------------------------------------------ shortest path
adha_status pdl_solve(uint32_t k, uint32_t C, const double *T, const double *R, const double *R0,
                      std::vector<uint32_t> *path, double *cost) {
  std::vector<double> dist(C), nd(C);
  std::vector<uint32_t> back((size_t)k * C, 0);
  for (uint32_t c = 0; c < C; ++c) dist[c] = (R0 ? R0[c] : 0.0) + T[c];
  for (uint32_t s = 1; s < k; ++s) {
    for (uint32_t b = 0; b < C; ++b) {
      double best = 0.0;
      uint32_t arg = 0;
      for (uint32_t a = 0; a < C; ++a) {
        const double v = dist[a] + (a == b ? 0.0 : R[(size_t)a * C + b]);
        if (a == 0 || v < best) {
          best = v;
          arg = a;
        }
      }
      nd[b] = best + T[(size_t)s * C + b];
      back[(size_t)s * C + b] = arg;
    }
    dist.swap(nd);
  }
  uint32_t end = 0;
  for (uint32_t c = 1; c < C; ++c)
    if (dist[c] < dist[end]) end = c;
  path->assign(k, 0);
  (*path)[k - 1] = end;
  for (uint32_t s = k - 1; s > 0; --s) (*path)[s - 1] = back[(size_t)s * C + (*path)[s]];
  *cost = dist[end];
  return ADHA_OK;
}

// ------------------------------------------------------------------ catalogue
static const uint32_t kAosoaTile = 64;

static void catalogue(const Shape &sh, const std::vector<SectionDesc> &secs, bool full, uint32_t cap,
                      std::vector<LayoutDesc> *out) {
  std::vector<LayoutDesc> all{layout_aos(sh), layout_soa(sh)};
  if (full) {
    all.push_back(layout_aos(sh, kAosoaTile));
    for (size_t i = 0; i < secs.size(); ++i)
      for (size_t j = i; j < secs.size(); ++j) {
        auto parts = ods_parts(secs, i, j, sh, cap);
        all.push_back(layout_from_parts(sh, parts, 1));
        all.push_back(layout_from_parts(sh, parts, kAosoaTile));
      }
  }
  for (auto &L : all) {
    bool dup = false;
    for (auto &M : *out)
      if (M.same_map(L)) dup = true;
    if (!dup) out->push_back(L);
  }
}

// ------------------------------------------------------------------ costs
// Analytic model: effective HBM bytes per record over a bandwidth.
// bytes one random access fetches: the 128-byte line (measured with the
// library's random-access probe: a 4-byte and a 128-byte random load run at
// nearly the same rate, and the counters read 128 bytes fetched per access)
static const double kGranule = 128.0;
static const double kBytesPerUs = 5.6e6;   // 70% of 8 TB/s
static const double kLaunchUs = 4.0;

static double group_stream_bytes(const LayoutDesc &l, size_t gi, const std::vector<int32_t> &touched) {
  const Group &g = l.groups[gi];
  double b = 0.0;
  for (int f : touched)
    if (l.group_of[f] == gi) b += std::max<double>(l.shape.ebytes[f], kGranule / g.T);
  return std::min<double>(b, g.S);
}

static double group_random_bytes(const LayoutDesc &l, size_t gi, const std::vector<int32_t> &touched) {
  const Group &g = l.groups[gi];
  if (g.T == 1 && g.fields.size() > 1) {
    uint32_t lo = ~0u, hi = 0;
    for (int f : touched)
      if (l.group_of[f] == gi) {
        lo = std::min(lo, l.p[f]);
        hi = std::max(hi, l.p[f] + l.shape.ebytes[f]);
      }
    if (hi == 0) return 0.0;
    return (hi - lo) + kGranule - 1.0;
  }
  double b = 0.0;
  for (int f : touched)
    if (l.group_of[f] == gi) b += l.shape.ebytes[f] + kGranule - 1.0;
  return b;
}

double analytic_bytes_per_record(const SectionDesc &s, const LayoutDesc &l) {
  double b = 0.0;
  const std::vector<int32_t> streamed = s.streamed_reads();
  // a stencil's neighbours are the record's own neighbourhood, served from
  // cache after the first touch: it moves the bytes of a direct pass
  const bool stream = s.degree == 0 || s.stencil;
  for (size_t gi = 0; gi < l.groups.size(); ++gi) {
    if (stream) b += group_stream_bytes(l, gi, streamed);
    else b += s.degree * group_random_bytes(l, gi, s.rd);
    b += group_stream_bytes(l, gi, s.wr);
  }
  if (s.degree && !s.stencil) b += 4.0 * s.degree;
  return b;
}

double analytic_section_us(const SectionDesc &s, const LayoutDesc &l) {
  return kLaunchUs + (double)l.shape.n * analytic_bytes_per_record(s, l) / kBytesPerUs;
}

// Bytes a remap a -> b moves when the groups the layouts share stay in
// place: 2 * N * (element bytes of the fields whose group changes).
double moving_bytes(const LayoutDesc &a, const LayoutDesc &b) {
  double e = 0.0;
  for (int f : moving_fields(a, b)) e += a.shape.ebytes[f];
  return 2.0 * (double)a.shape.n * e;
}

double analytic_remap_us(const LayoutDesc &a, const LayoutDesc &b, bool whole) {
  if (a.same_groups(b)) return 0.0;
  const double bytes = whole ? 2.0 * (double)a.shape.n * a.shape.record_bytes() : moving_bytes(a, b);
  return kLaunchUs + bytes / kBytesPerUs;
}

// Median time in microseconds of `reps` runs of fn on `stream`, after one
// warm-up.  With long_us > 0 and reps == 1 the warm-up is timed as well, and
// a warm-up of at least long_us is the figure (the timed run would repeat a
// launch whose one-time costs are small next to it).
template <class Fn>
static adha_status time_us(hipStream_t stream, uint32_t reps, Fn fn, double *out, double long_us = 0.0) {
  hipEvent_t a, b;
  ADHA_HIP(hipEventCreate(&a));
  ADHA_HIP(hipEventCreate(&b));
  std::vector<double> ts;
  const bool time_warm = long_us > 0.0 && reps == 1;
  if (time_warm) (void)hipEventRecord(a, stream);
  adha_status st = fn();
  if (time_warm && st >= 0) {
    (void)hipEventRecord(b, stream);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (ms * 1000.0 >= long_us) {
      ts.push_back(ms * 1000.0);
      reps = 0;
    }
  }
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

// Section timings of one launch (reps = 1) take a warm-up of at least this
// long as the figure.
static const double kLongLaunchUs = 2000.0;

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  adha_status alloc(size_t n) {
    if (hipMalloc(&p, std::max<size_t>(n, 256)) != hipSuccess) {
      p = nullptr;
      return fail(ADHA_ERR_OOM, "device scratch of %zu bytes failed", n);
    }
    return ADHA_OK;
  }
};

// Which section times measured_costs takes on the device (the remap figure
// is always measured).
enum TimeSections { kTimeAll, kTimeNone, kTimeUntrained };

// Section s and the groups of l that hold a field it touches (read, written
// or its key): their fields, tiles and the offsets of the touched fields.
static std::vector<uint64_t> touched_groups_key(size_t s, const SectionDesc &d, const LayoutDesc &l) {
  std::vector<int32_t> t = d.streamed_reads();
  t.insert(t.end(), d.wr.begin(), d.wr.end());
  std::vector<uint32_t> gs;
  for (int f : t) gs.push_back(l.group_of[f]);
  std::sort(gs.begin(), gs.end());
  gs.erase(std::unique(gs.begin(), gs.end()), gs.end());
  // (and whether the layout fits 32-bit offsets, which some kernel forms need)
  std::vector<uint64_t> key{(uint64_t)s, l.nbytes <= (1ull << 32) ? 1u : 0u};
  for (uint32_t g : gs) {
    const Group &G = l.groups[g];
    key.push_back(((uint64_t)G.T << 32) | G.fields.size());
    for (int f : G.fields) key.push_back((uint64_t)f);
  }
  return key;
}
// How remap costs are measured: every pair as an in-place remap (the placed
// executor), one whole-struct figure for every pair (the two-buffer
// executors), or that figure scaled by the bytes each in-place remap moves.
enum RemapCosts { kRemapPairs, kRemapWhole, kRemapScaled };

static adha_status measured_costs(Ctx *ctx, const Shape &sh, const std::vector<SectionDesc> &secs,
                                  const std::vector<adha_layout *> &cands, uint32_t reps,
                                  const int32_t *idx_in, uint64_t idx_count, hipStream_t stream,
                                  std::vector<double> *T, std::vector<double> *R, TimeSections which = kTimeAll,
                                  RemapCosts rmode = kRemapPairs, const std::vector<char> *only = nullptr) {
  // only: time just the (section, candidate) entries it marks, leave R alone
  const size_t k = secs.size(), C = cands.size();
  const bool sections = which != kTimeNone || only;
  uint64_t maxb = 0;
  uint32_t maxd = 0;
  for (auto *l : cands) maxb = std::max(maxb, l->d.nbytes);
  for (auto &s : secs) maxd = std::max(maxd, s.degree);
  DevBuf a, b, ix, tab;
  ADHA_TRY(a.alloc(maxb));
  ADHA_TRY(b.alloc(maxb));
  // reductions write their tables here while being timed, not into the
  // caller's result arrays
  ADHA_TRY(tab.alloc(ADHA_MAX_REDUCE_CELLS * 8));
  ADHA_HIP(hipMemsetAsync(a.p, 0, maxb, stream));
  const int32_t *idx = idx_in;
  if (sections && maxd > 0 && sh.n > 0 && (!idx_in || idx_count < (uint64_t)sh.n * maxd)) {
    ADHA_TRY(ix.alloc((size_t)sh.n * maxd * 4));
    ADHA_TRY(fill_uniform_index((int32_t *)ix.p, (uint64_t)sh.n * maxd, sh.n, 0x5eedULL, stream));
    idx = (const int32_t *)ix.p;
  }
  if (which == kTimeAll && !only) T->assign(k * C, 0.0);
  // a section's time depends on the groups holding the fields it touches
  // (their fields and tiles), not on the rest of the layout: time each such
  // arrangement once per section
  std::map<std::vector<uint64_t>, double> seen;
  for (size_t c = 0; c < C && sections; ++c)
    for (size_t s = 0; s < k; ++s) {
      if (only ? !(*only)[s * C + c] : (which == kTimeUntrained && secs[s].op != ADHA_OP_REDUCE && !secs[s].stencil))
        continue;
      const std::vector<uint64_t> key = touched_groups_key(s, secs[s], cands[c]->d);
      auto it = seen.find(key);
      if (it != seen.end()) {
        (*T)[s * C + c] = it->second;
        continue;
      }
      // a gather section's index array is [N][d]; a wider one is read as [N][d] too
      ADHA_TRY(time_us(stream, reps,
                       [&] { return section_launch(ctx, secs[s], cands[c]->d, a.p, idx, stream, tab.p); },
                       &(*T)[s * C + c], kLongLaunchUs));
      seen.emplace(key, (*T)[s * C + c]);
    }
  if (only) {
    ADHA_HIP(hipStreamSynchronize(stream));
    return ADHA_OK;
  }
  R->assign(C * C, 0.0);
  if (rmode == kRemapWhole || rmode == kRemapScaled) {
    // whole-struct remaps (two buffers): one measured figure, from a few
    // representative pairs, serves every pair of different layouts
    double rsum = 0.0;
    int rn = 0;
    for (size_t c = 1; c < C && rn < 4; ++c) {
      double t = 0.0;
      ADHA_TRY(time_us(stream, reps, [&] { return remap_one(ctx, cands[0], a.p, cands[c], b.p, stream); }, &t));
      rsum += t;
      ++rn;
    }
    const double rem = rn ? rsum / rn : 0.0;
    // scaled: that figure spread over the bytes each in-place remap moves
    const double whole_bytes = 2.0 * (double)sh.n * sh.record_bytes();
    for (size_t x = 0; x < C; ++x)
      for (size_t y = 0; y < C; ++y) {
        if (cands[x]->d.same_groups(cands[y]->d)) continue;
        if (rmode == kRemapWhole) {
          (*R)[x * C + y] = rem;
        } else {
          const double frac = whole_bytes > 0 ? moving_bytes(cands[x]->d, cands[y]->d) / whole_bytes : 0.0;
          (*R)[x * C + y] = kLaunchUs + std::max(0.0, rem - kLaunchUs) * frac;
        }
      }
  } else {
    // in-place remaps: every ordered pair timed as the placed executor runs
    // it (the first layout at its canonical bases, the groups the second
    // shares with it kept there, the others placed after)
    DevBuf arena;
    uint64_t need = 0;
    std::vector<LayoutDesc> pl2;
    for (size_t x = 0; x < C; ++x)
      for (size_t y = 0; y < C; ++y) {
        if (x == y) continue;
        uint64_t ab = 0;
        place_sequence({&cands[x]->d, &cands[y]->d}, &pl2, &ab);
        need = std::max(need, ab);
      }
    if (need) ADHA_TRY(arena.alloc(need));
    for (size_t x = 0; x < C; ++x)
      for (size_t y = 0; y < C; ++y) {
        if (x == y || cands[x]->d.same_groups(cands[y]->d)) continue;
        uint64_t ab = 0;
        place_sequence({&cands[x]->d, &cands[y]->d}, &pl2, &ab);
        double t = 0.0;
        ADHA_TRY(time_us(stream, reps, [&] { return remap_in_place(ctx, pl2[0], pl2[1], arena.p, stream); }, &t));
        (*R)[x * C + y] = t;
      }
  }
  ADHA_HIP(hipStreamSynchronize(stream));
  return ADHA_OK;
}

// ------------------------------------------------------------------ structured flow
static const uint32_t kNoJoin = 0xFFFFFFFFu;

// A block of a structured program: a section, a sequence of blocks, or a
// two-way branch over two sequences.
struct FlowBlock {
  int kind = 0;            // 0 section, 1 sequence, 2 branch
  int sec = -1;            // section
  std::vector<int> items;  // sequence
  int first = -1, second = -1, branch = -1;  // branch: its two sequences and its index
  double p = 0.0;
};

// Parses a token list into blocks (block 0 is the root sequence).
static adha_status parse_flow(const std::vector<int32_t> &tok, const std::vector<double> &probs, size_t k,
                              std::vector<FlowBlock> *blocks) {
  blocks->clear();
  blocks->push_back(FlowBlock{1});
  std::vector<int> stack{0};          // open sequences
  std::vector<int> open_branch;       // open branches
  std::vector<char> seen(k, 0);
  int n_if = 0;
  for (size_t t = 0; t < tok.size(); ++t) {
    const int32_t x = tok[t];
    if (x >= 0) {
      if ((size_t)x >= k) return fail(ADHA_ERR_INVALID, "token %zu names section %d of %zu", t, x, k);
      if (seen[x]) return fail(ADHA_ERR_INVALID, "section %d appears twice in the flow", x);
      seen[x] = 1;
      FlowBlock b;
      b.kind = 0;
      b.sec = x;
      blocks->push_back(b);
      (*blocks)[stack.back()].items.push_back((int)blocks->size() - 1);
    } else if (x == ADHA_TOK_IF) {
      if (n_if >= (int)probs.size()) return fail(ADHA_ERR_INVALID, "more branches than probabilities");
      const double p = probs[n_if];
      if (!(p >= 0.0 && p <= 1.0)) return fail(ADHA_ERR_INVALID, "branch %d probability %g not in [0, 1]", n_if, p);
      FlowBlock br;
      br.kind = 2;
      br.p = p;
      br.branch = n_if++;
      blocks->push_back(br);
      const int bid = (int)blocks->size() - 1;
      (*blocks)[stack.back()].items.push_back(bid);
      blocks->push_back(FlowBlock{1});
      (*blocks)[bid].first = (int)blocks->size() - 1;
      blocks->push_back(FlowBlock{1});
      (*blocks)[bid].second = (int)blocks->size() - 1;
      open_branch.push_back(bid);
      stack.push_back((*blocks)[bid].first);
    } else if (x == ADHA_TOK_ELSE) {
      if (open_branch.empty()) return fail(ADHA_ERR_INVALID, "ELSE outside a branch at token %zu", t);
      const FlowBlock &br = (*blocks)[open_branch.back()];
      if (stack.back() != br.first) return fail(ADHA_ERR_INVALID, "second ELSE in one branch at token %zu", t);
      stack.back() = br.second;
    } else if (x == ADHA_TOK_END) {
      if (open_branch.empty()) return fail(ADHA_ERR_INVALID, "END outside a branch at token %zu", t);
      open_branch.pop_back();
      stack.pop_back();
    } else {
      return fail(ADHA_ERR_INVALID, "unknown token %d", x);
    }
  }
  if (!open_branch.empty()) return fail(ADHA_ERR_INVALID, "a branch is not closed");
  if (n_if != (int)probs.size()) return fail(ADHA_ERR_INVALID, "%d branches but %zu probabilities", n_if, probs.size());
  for (size_t x = 0; x < k; ++x)
    if (!seen[x]) return fail(ADHA_ERR_INVALID, "section %zu is not in the flow", x);
  return ADHA_OK;
}

// Expected-cost shortest path over a structured program: every block gets
// an M x M matrix B[a][b], the least expected cost of running it entered in
// node a and left in node b.  A section s: R[a][b] + T[s][b].  A sequence:
// the min-plus product of its blocks' matrices (empty: 0 on the diagonal).
// A branch taken with probability p: p * min_x (B1[a][x] + R[x][b]) +
// (1 - p) * min_y (B2[a][y] + R[y][b]) -- each part may end in its own
// node and moves to the join node b.  The program: min over a, b of
// R0[a] + B_root[a][b].  Ties go to the smaller node index.
struct FlowSolver {
  size_t M;
  const double *T, *R;
  const std::vector<FlowBlock> &blocks;
  std::vector<std::vector<double>> mat;
  std::vector<std::vector<std::vector<uint32_t>>> seq_arg;  // per sequence: per step a..c -> middle
  std::vector<std::vector<uint32_t>> arg1, arg2;            // per branch block
  double r(size_t a, size_t b) const { return a == b ? 0.0 : R[a * M + b]; }

  FlowSolver(size_t m, const double *t, const double *rr, const std::vector<FlowBlock> &b)
      : M(m), T(t), R(rr), blocks(b), mat(b.size()), seq_arg(b.size()), arg1(b.size()), arg2(b.size()) {}

  void solve(int id) {
    const FlowBlock &b = blocks[id];
    const double inf = std::numeric_limits<double>::infinity();
    std::vector<double> &B = mat[id];
    B.assign(M * M, inf);
    if (b.kind == 0) {
      for (size_t a = 0; a < M; ++a)
        for (size_t c = 0; c < M; ++c) B[a * M + c] = r(a, c) + T[(size_t)b.sec * M + c];
    } else if (b.kind == 1) {
      if (b.items.empty()) {
        for (size_t a = 0; a < M; ++a) B[a * M + a] = 0.0;
        return;
      }
      for (int c : b.items) solve(c);
      B = mat[b.items[0]];
      for (size_t i = 1; i < b.items.size(); ++i) {
        const std::vector<double> &N = mat[b.items[i]];
        std::vector<double> P(M * M, inf);
        std::vector<uint32_t> arg(M * M, 0);
        for (size_t a = 0; a < M; ++a)
          for (size_t c = 0; c < M; ++c) {
            double best = inf;
            uint32_t bm = 0;
            for (size_t m = 0; m < M; ++m) {
              const double v = B[a * M + m] + N[m * M + c];
              if (v < best) {
                best = v;
                bm = (uint32_t)m;
              }
            }
            P[a * M + c] = best;
            arg[a * M + c] = bm;
          }
        B.swap(P);
        seq_arg[id].push_back(std::move(arg));
      }
    } else {
      solve(b.first);
      solve(b.second);
      const std::vector<double> &B1 = mat[b.first], &B2 = mat[b.second];
      arg1[id].assign(M * M, 0);
      arg2[id].assign(M * M, 0);
      for (size_t a = 0; a < M; ++a)
        for (size_t c = 0; c < M; ++c) {
          double b1 = inf, b2 = inf;
          uint32_t x1 = 0, x2 = 0;
          for (size_t x = 0; x < M; ++x) {
            const double v1 = B1[a * M + x] + r(x, c), v2 = B2[a * M + x] + r(x, c);
            if (v1 < b1) b1 = v1, x1 = (uint32_t)x;
            if (v2 < b2) b2 = v2, x2 = (uint32_t)x;
          }
          // a part that never runs (p = 0 or 1) adds nothing
          const double e = (b.p > 0.0 ? b.p * b1 : 0.0) + (b.p < 1.0 ? (1.0 - b.p) * b2 : 0.0);
          B[a * M + c] = e;
          arg1[id][a * M + c] = x1;
          arg2[id][a * M + c] = x2;
        }
    }
  }

  // Node of every section and the join node of every branch, for block id
  // entered in a and left in c.
  void rebuild(int id, uint32_t a, uint32_t c, std::vector<uint32_t> *node, std::vector<uint32_t> *join) const {
    const FlowBlock &b = blocks[id];
    if (b.kind == 0) {
      (*node)[b.sec] = c;
    } else if (b.kind == 1) {
      if (b.items.empty()) return;
      uint32_t exit = c;
      for (size_t i = b.items.size() - 1; i >= 1; --i) {
        const uint32_t mid = seq_arg[id][i - 1][(size_t)a * M + exit];
        rebuild(b.items[i], mid, exit, node, join);
        exit = mid;
      }
      rebuild(b.items[0], a, exit, node, join);
    } else {
      (*join)[b.branch] = c;
      rebuild(b.first, a, arg1[id][(size_t)a * M + c], node, join);
      rebuild(b.second, a, arg2[id][(size_t)a * M + c], node, join);
    }
  }
};

static adha_status flow_solve(size_t k, size_t M, const double *T, const double *R, const double *R0,
                              const std::vector<FlowBlock> &blocks, size_t n_branch, std::vector<uint32_t> *node,
                              std::vector<uint32_t> *join, double *cost, uint32_t *start = nullptr) {
  FlowSolver f(M, T, R, blocks);
  f.solve(0);
  const std::vector<double> &B = f.mat[0];
  double best = std::numeric_limits<double>::infinity();
  uint32_t ba = 0, bc = 0;
  for (size_t a = 0; a < M; ++a)
    for (size_t c = 0; c < M; ++c) {
      const double v = (R0 ? R0[a] : 0.0) + B[a * M + c];
      if (v < best) best = v, ba = (uint32_t)a, bc = (uint32_t)c;
    }
  node->assign(k, 0);
  join->assign(n_branch, 0);
  f.rebuild(0, ba, bc, node, join);
  *cost = best;
  if (start) *start = ba;
  return ADHA_OK;
}

// The GPU's whole-struct remap figure of a plan: every pair of different
// layouts costs the same (zero when the plan has one candidate).
static double device_remap_figure(const adha_plan *pl) {
  const size_t C = pl->cands.size();
  return C > 1 ? pl->R[0 * C + 1] : 0.0;
}

// The node graph of a plan over both devices: node m is (device m / C,
// layout m % C).  T is k*M, R is M*M.
static void node_tables(const adha_plan *pl, std::vector<double> *T, std::vector<double> *R) {
  const size_t k = pl->secs.size(), C = pl->cands.size(), M = pl->hetero ? 2 * C : C;
  T->assign(k * M, 0.0);
  R->assign(M * M, 0.0);
  for (size_t s = 0; s < k; ++s)
    for (size_t m = 0; m < M; ++m) (*T)[s * M + m] = m < C ? pl->T[s * C + m] : pl->TH[s * C + m - C];
  const double rd = device_remap_figure(pl);
  for (size_t x = 0; x < M; ++x)
    for (size_t y = 0; y < M; ++y) {
      const size_t a = x % C, b = y % C;
      const bool gx = x < C, gy = y < C;
      double r;
      if (gx && gy) r = pl->R[a * C + b];
      else if (!gx && !gy) r = a == b ? 0.0 : pl->rem_h;
      else r = (gx ? pl->xfer_dh : pl->xfer_hd) + (a == b ? 0.0 : rd);
      (*R)[x * M + y] = x == y ? 0.0 : r;
    }
}

// Host costs analytic: the bytes model over a host bandwidth, plus thread
// start-up; transfers over PCIe.
static const double kHostBytesPerUs = 4.0e4;  // 40 GB/s over the host cores
static const double kHostStartUs = 30.0;
static const double kPcieBytesPerUs = 5.0e4;  // 50 GB/s each way
static const double kCopyStartUs = 10.0;

static void analytic_host_costs(adha_plan *pl) {
  const size_t k = pl->secs.size(), C = pl->cands.size();
  pl->TH.assign(k * C, 0.0);
  for (size_t s = 0; s < k; ++s)
    for (size_t c = 0; c < C; ++c)
      pl->TH[s * C + c] = kHostStartUs + (double)pl->shape.n * analytic_bytes_per_record(pl->secs[s], pl->cands[c]->d) /
                                             kHostBytesPerUs;
  const double bytes = (double)pl->shape.n * pl->shape.record_bytes();
  pl->rem_h = kHostStartUs + 2.0 * bytes / kHostBytesPerUs;
  pl->xfer_dh = pl->xfer_hd = kCopyStartUs + bytes / kPcieBytesPerUs;
}

// Host costs measured: each (section, candidate) on host scratch with the
// context's host threads (median of reps after one warm-up), one host
// remap, and a pinned transfer each way of the whole struct.
static adha_status measured_host_costs(Ctx *ctx, adha_plan *pl, uint32_t reps, const int32_t *idx_dev,
                                       uint64_t idx_count, hipStream_t stream) {
  const size_t k = pl->secs.size(), C = pl->cands.size();
  const Shape &sh = pl->shape;
  const uint32_t threads = host_threads(ctx);
  uint64_t maxb = 256;
  uint32_t maxd = 0;
  for (auto *l : pl->cands) maxb = std::max(maxb, l->d.nbytes);
  for (auto &s : pl->secs) maxd = std::max(maxd, s.degree);
  std::vector<uint8_t> a(maxb, 0), b(maxb, 0);
  std::vector<int32_t> idx;
  if (maxd > 0 && sh.n > 0) {
    idx.resize((size_t)sh.n * maxd);
    if (idx_dev && idx_count >= (uint64_t)sh.n * maxd) {
      ADHA_HIP(hipMemcpy(idx.data(), idx_dev, idx.size() * 4, hipMemcpyDeviceToHost));
    } else {
      for (size_t i = 0; i < idx.size(); ++i) {  // uniform neighbours (SplitMix64, multiply-shift)
        uint64_t z = ((0x5eedULL << 32) + i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        idx[i] = (int32_t)(((z >> 32) * (uint64_t)sh.n) >> 32);
      }
    }
  }
  std::vector<uint64_t> table(ADHA_MAX_REDUCE_CELLS, 0);
  auto median_us = [&](auto fn) {
    fn();
    std::vector<double> ts;
    for (uint32_t r = 0; r < std::max<uint32_t>(1, reps); ++r) {
      auto t0 = std::chrono::steady_clock::now();
      fn();
      ts.push_back(std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count());
    }
    std::sort(ts.begin(), ts.end());
    return ts[ts.size() / 2];
  };
  pl->TH.assign(k * C, 0.0);
  for (size_t c = 0; c < C; ++c)
    for (size_t s = 0; s < k; ++s)
      pl->TH[s * C + c] = median_us([&] {
        uint64_t bad = 0;
        (void)host_section_run(threads, pl->secs[s], pl->cands[c]->d, a.data(), idx.data(), table.data(), &bad);
      });
  pl->rem_h = C > 1 ? median_us([&] { (void)host_remap(threads, pl->cands[0]->d, a.data(), pl->cands[1]->d, b.data()); })
                    : 0.0;
  // transfers: pinned host staging and device scratch of the struct's size
  const uint64_t bytes = pl->cands[0]->d.nbytes;
  void *hp = nullptr, *dp = nullptr;
  if (bytes) {
    ADHA_HIP(hipHostMalloc(&hp, bytes, hipHostMallocDefault));
    if (hipMalloc(&dp, bytes) != hipSuccess) {
      (void)hipHostFree(hp);
      return fail(ADHA_ERR_OOM, "device scratch of %llu bytes failed", (unsigned long long)bytes);
    }
    pl->xfer_dh = median_us([&] {
      (void)hipMemcpyAsync(hp, dp, bytes, hipMemcpyDeviceToHost, stream);
      (void)hipStreamSynchronize(stream);
    });
    pl->xfer_hd = median_us([&] {
      (void)hipMemcpyAsync(dp, hp, bytes, hipMemcpyHostToDevice, stream);
      (void)hipStreamSynchronize(stream);
    });
    (void)hipFree(dp);
    (void)hipHostFree(hp);
  }
  return ADHA_OK;
}

// The plan's placed sequence: the start layout at its canonical bases, then
// each section's layout with the groups the previous one shares kept in
// place (place_sequence), and the arena they need.
static adha_status place_plan(adha_plan *pl, const LayoutDesc &start) {
  for (auto *l : pl->placed) delete l;
  pl->placed.clear();
  std::vector<const LayoutDesc *> seq{&start};
  for (uint32_t c : pl->choice) seq.push_back(&pl->cands[c]->d);
  std::vector<LayoutDesc> out;
  place_sequence(seq, &out, &pl->arena);
  for (auto &L : out) {
    adha_layout *l = new_layout(std::move(L));
    if (!l) return fail(ADHA_ERR_OOM, "layout allocation failed");
    pl->placed.push_back(l);
  }
  return ADHA_OK;
}

}  // namespace adha

using namespace adha;

extern "C" {

adha_status adha_program_create(const adha_struct *s, uint32_t k, const adha_section *const *secs,
                                adha_program **out) {
  if (!s || !out || (k && !secs)) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (k == 0 || k > ADHA_MAX_SECTIONS) return fail(ADHA_ERR_INVALID, "k = %u not in [1, %d]", k, ADHA_MAX_SECTIONS);
  auto *p = new (std::nothrow) adha_program;
  if (!p) return fail(ADHA_ERR_OOM, "program allocation failed");
  p->shape = s->shape;
  for (uint32_t i = 0; i < k; ++i) {
    if (!secs[i] || !secs[i]->d.shape.same(s->shape)) {
      delete p;
      return fail(ADHA_ERR_INVALID, "section %u is NULL or belongs to another struct", i);
    }
    p->secs.push_back(secs[i]->d);
  }
  *out = p;
  return ADHA_OK;
}

adha_status adha_program_destroy(adha_program *p) {
  delete p;
  return ADHA_OK;
}

adha_status adha_program_set_flow(adha_program *p, uint32_t n_tokens, const int32_t *tokens, const double *probs) {
  if (!p) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (n_tokens == 0) {
    p->tokens.clear();
    p->probs.clear();
    return ADHA_OK;
  }
  if (!tokens) return fail(ADHA_ERR_INVALID, "tokens is NULL");
  std::vector<int32_t> tok(tokens, tokens + n_tokens);
  size_t n_if = 0;
  for (int32_t x : tok) n_if += x == ADHA_TOK_IF;
  if (n_if && !probs) return fail(ADHA_ERR_INVALID, "probs is NULL");
  std::vector<double> pr(probs, probs + n_if);
  std::vector<FlowBlock> blocks;
  ADHA_TRY(parse_flow(tok, pr, p->secs.size(), &blocks));
  p->tokens = std::move(tok);
  p->probs = std::move(pr);
  return ADHA_OK;
}

adha_status adha_affinity(const adha_program *p, uint32_t first, uint32_t last, uint64_t *w) {
  if (!p || !w) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (first > last || last >= p->secs.size()) return fail(ADHA_ERR_INVALID, "bad section range");
  auto v = affinity(p->secs, first, last, p->shape.nfields());
  memcpy(w, v.data(), v.size() * sizeof(uint64_t));
  return ADHA_OK;
}

adha_status adha_ods(const adha_program *p, uint32_t first, uint32_t last, uint32_t cap_bytes, uint32_t tile,
                     adha_layout **out) {
  if (!p || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (first > last || last >= p->secs.size()) return fail(ADHA_ERR_INVALID, "bad section range");
  if (tile == 0 || tile > ADHA_MAX_TILE || (tile & (tile - 1))) return fail(ADHA_ERR_INVALID, "bad tile %u", tile);
  auto parts = ods_parts(p->secs, first, last, p->shape, cap_bytes);
  adha_layout *l = new_layout(layout_from_parts(p->shape, parts, tile));
  if (!l) return fail(ADHA_ERR_OOM, "layout allocation failed");
  *out = l;
  return ADHA_OK;
}

adha_status adha_pdl_solve(uint32_t k, uint32_t C, const double *T, const double *R, const double *R0,
                           uint32_t *path, double *cost) {
  if (!T || !R || !path || !cost) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (k == 0 || C == 0) return fail(ADHA_ERR_INVALID, "k and C must be positive");
  std::vector<uint32_t> pv;
  double c = 0;
  ADHA_TRY(pdl_solve(k, C, T, R, R0, &pv, &c));
  memcpy(path, pv.data(), k * sizeof(uint32_t));
  *cost = c;
  return ADHA_OK;
}

adha_status adha_flow_solve(uint32_t k, uint32_t C, const double *T, const double *R, const double *R0,
                            uint32_t n_tokens, const int32_t *tokens, const double *probs, uint32_t *node,
                            uint32_t *join, uint32_t *start, double *cost) {
  if (!T || !R || !tokens || !node || !cost) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (k == 0 || C == 0) return fail(ADHA_ERR_INVALID, "k and C must be positive");
  std::vector<int32_t> tok(tokens, tokens + n_tokens);
  size_t n_if = 0;
  for (int32_t x : tok) n_if += x == ADHA_TOK_IF;
  if (n_if && (!probs || !join)) return fail(ADHA_ERR_INVALID, "branches need probs and join");
  std::vector<double> pr(probs ? probs : nullptr, probs ? probs + n_if : nullptr);
  std::vector<FlowBlock> blocks;
  ADHA_TRY(parse_flow(tok, pr, k, &blocks));
  std::vector<uint32_t> nv, jv;
  double c = 0;
  uint32_t a = 0;
  ADHA_TRY(flow_solve(k, C, T, R, R0, blocks, n_if, &nv, &jv, &c, &a));
  memcpy(node, nv.data(), k * sizeof(uint32_t));
  if (n_if) memcpy(join, jv.data(), n_if * sizeof(uint32_t));
  if (start) *start = a;
  *cost = c;
  return ADHA_OK;
}

adha_status adha_plan_opts_default(adha_plan_opts *o) {
  if (!o) return fail(ADHA_ERR_INVALID, "NULL argument");
  o->cost = ADHA_COST_MEASURED;
  o->catalogue = ADHA_CAT_FULL;
  o->cap_bytes = 128;  // one 128-byte line: a gathered structure comes in one access
  o->init = ADHA_INIT_FREE;
  o->reps = 5;
  o->devices = ADHA_DEVICES_GPU;
  o->pair_remaps = 1;
  o->verify_rounds = 0;
  return ADHA_OK;
}

adha_status adha_plan_create(adha_ctx *ctx, const adha_program *p, const adha_plan_opts *o,
                             const int32_t *idx, uint64_t idx_count, void *stream, adha_plan **out) {
  if (!p || !o || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  // the option fields' enums are checked as integers before any other use
  const int32_t cost = enum_value(o->cost), devices = enum_value(o->devices), init = enum_value(o->init);
  const int32_t catalogue_kind = enum_value(o->catalogue);
  if (cost < ADHA_COST_MEASURED || cost > ADHA_COST_LEARNED) return fail(ADHA_ERR_INVALID, "unknown cost source");
  if (catalogue_kind != ADHA_CAT_AOS_SOA && catalogue_kind != ADHA_CAT_FULL)
    return fail(ADHA_ERR_INVALID, "unknown catalogue %d", catalogue_kind);
  if (devices != ADHA_DEVICES_GPU && devices != ADHA_DEVICES_GPU_HOST)
    return fail(ADHA_ERR_INVALID, "unknown devices option %d", devices);
  if (init < ADHA_INIT_FREE || init > ADHA_INIT_HOST_AOS) return fail(ADHA_ERR_INVALID, "unknown init option");
  if (o->cost != ADHA_COST_ANALYTIC && !ctx) return fail(ADHA_ERR_INVALID, "measured and learned costs need a context");
  if (o->cap_bytes == 0) return fail(ADHA_ERR_INVALID, "cap_bytes must be positive");
  if (idx && ((uintptr_t)idx & 255u)) return fail(ADHA_ERR_INVALID, "idx is not 256-byte aligned");
  if (o->init == ADHA_INIT_HOST_AOS && o->devices != ADHA_DEVICES_GPU_HOST)
    return fail(ADHA_ERR_INVALID, "data starting on the host needs a plan over both devices");
  if (!p->tokens.empty() && o->devices != ADHA_DEVICES_GPU)
    return fail(ADHA_ERR_UNSUPPORTED, "programs with branches are planned for the GPU only");
  auto t0 = std::chrono::steady_clock::now();
  std::unique_ptr<adha_plan> pl(new (std::nothrow) adha_plan);
  if (!pl) return fail(ADHA_ERR_OOM, "plan allocation failed");
  pl->shape = p->shape;
  pl->secs = p->secs;
  std::vector<LayoutDesc> cat;
  catalogue(p->shape, p->secs, o->catalogue == ADHA_CAT_FULL, o->cap_bytes, &cat);
  for (auto &L : cat) {
    adha_layout *l = new_layout(L);
    if (!l) return fail(ADHA_ERR_OOM, "layout allocation failed");
    pl->cands.push_back(l);
  }
  const size_t k = p->secs.size(), C = pl->cands.size();
  // structured programs and plans over both devices run with the two-buffer
  // executors, which remap the whole struct; linear GPU plans run placed
  pl->whole = !p->tokens.empty() || o->devices == ADHA_DEVICES_GPU_HOST;
  adha_status result = ADHA_OK;
  adha_cost_source src = o->cost;
  hipStream_t st = (hipStream_t)stream;
  std::unique_ptr<DeviceGuard> guard;
  if (ctx) guard.reset(new DeviceGuard(ctx->c.device));
  if (src == ADHA_COST_LEARNED) {
    if (!ctx->c.has_model) {
      src = ADHA_COST_MEASURED;
      result = ADHA_WARN_FALLBACK;
    } else {
      std::vector<std::vector<float>> feats;
      std::vector<double> base;
      for (size_t s = 0; s < k; ++s)
        for (size_t c = 0; c < C; ++c) {
          std::vector<float> f(ADHA_N_FEATURES);
          section_features(p->secs[s], pl->cands[c]->d, f.data());
          feats.push_back(f);
          base.push_back(analytic_section_us(p->secs[s], pl->cands[c]->d));
        }
      std::vector<double> us;
      ADHA_TRY(predict_costs(&ctx->c, feats, base, &us, st));
      pl->T = us;
      // the network was trained on direct loops and index gathers;
      // reductions and stencils are timed on the device
      bool untrained = false;
      for (const SectionDesc &d : p->secs) untrained |= d.op == ADHA_OP_REDUCE || d.stencil;
      // remap weights: a few measured whole-struct remaps scaled by the
      // bytes each pair moves (milliseconds of device time, not the seconds
      // every pair would take)
      ADHA_TRY(measured_costs(&ctx->c, p->shape, p->secs, pl->cands, std::max<uint32_t>(1, o->reps), idx,
                              idx_count, st, &pl->T, &pl->R, untrained ? kTimeUntrained : kTimeNone,
                              pl->whole ? kRemapWhole : kRemapScaled));
      // verification: time the sections of the path the predictions choose,
      // put those times in the table and solve again, until the chosen
      // path is timed throughout (or the rounds run out)
      if (o->verify_rounds && p->tokens.empty() && o->devices == ADHA_DEVICES_GPU) {
        std::vector<char> known(k * C, 0);
        for (size_t s2 = 0; s2 < k; ++s2)
          if (p->secs[s2].op == ADHA_OP_REDUCE || p->secs[s2].stencil)
            for (size_t c = 0; c < C; ++c) known[s2 * C + c] = 1;
        const LayoutDesc aos = layout_aos(p->shape);
        std::vector<double> R0(C, 0.0);
        if (o->init == ADHA_INIT_AOS)
          for (size_t c = 0; c < C; ++c) R0[c] = pl->R[0 * C + c];
        for (uint32_t round = 0; round < o->verify_rounds; ++round) {
          std::vector<uint32_t> path;
          double cst = 0.0;
          ADHA_TRY(pdl_solve((uint32_t)k, (uint32_t)C, pl->T.data(), pl->R.data(), R0.data(), &path, &cst));
          std::vector<char> want(k * C, 0);
          bool any = false;
          for (size_t s2 = 0; s2 < k; ++s2)
            if (!known[s2 * C + path[s2]]) want[s2 * C + path[s2]] = any = true;
          if (!any) break;
          ADHA_TRY(measured_costs(&ctx->c, p->shape, p->secs, pl->cands, std::max<uint32_t>(1, o->reps), idx,
                                  idx_count, st, &pl->T, &pl->R, kTimeNone, kRemapScaled, &want));
          for (size_t e = 0; e < k * C; ++e)
            if (want[e]) {
              known[e] = 1;
              ++pl->verified;
            }
        }
      }
    }
  }
  if (src == ADHA_COST_ANALYTIC) {
    pl->T.resize(k * C);
    pl->R.resize(C * C);
    for (size_t s = 0; s < k; ++s)
      for (size_t c = 0; c < C; ++c) pl->T[s * C + c] = analytic_section_us(p->secs[s], pl->cands[c]->d);
    for (size_t a = 0; a < C; ++a)
      for (size_t b = 0; b < C; ++b)
        pl->R[a * C + b] = analytic_remap_us(pl->cands[a]->d, pl->cands[b]->d, pl->whole);
  } else if (src == ADHA_COST_MEASURED) {
    ADHA_TRY(measured_costs(&ctx->c, p->shape, p->secs, pl->cands, std::max<uint32_t>(1, o->reps), idx,
                            idx_count, st, &pl->T, &pl->R, kTimeAll,
                            pl->whole ? kRemapWhole : (o->pair_remaps ? kRemapPairs : kRemapScaled)));
  }
  if (o->devices == ADHA_DEVICES_GPU_HOST) {
    pl->hetero = true;
    if (o->cost == ADHA_COST_ANALYTIC) analytic_host_costs(pl.get());
    else ADHA_TRY(measured_host_costs(&ctx->c, pl.get(), std::max<uint32_t>(1, o->reps), idx, idx_count, st));
  }
  std::vector<double> NT, NR;
  node_tables(pl.get(), &NT, &NR);
  const size_t M = pl->hetero ? 2 * C : C;
  std::vector<double> R0(M, 0.0);
  if (o->init == ADHA_INIT_AOS)
    for (size_t m = 0; m < M; ++m) R0[m] = NR[0 * M + m];
  if (o->init == ADHA_INIT_HOST_AOS)
    for (size_t m = 0; m < M; ++m) R0[m] = m == C ? 0.0 : NR[C * M + m];
  std::vector<uint32_t> nodes;
  if (p->tokens.empty()) {
    ADHA_TRY(pdl_solve((uint32_t)k, (uint32_t)M, NT.data(), NR.data(), R0.data(), &nodes, &pl->cost));
  } else {
    std::vector<FlowBlock> blocks;
    ADHA_TRY(parse_flow(p->tokens, p->probs, k, &blocks));
    pl->tokens = p->tokens;
    pl->probs = p->probs;
    ADHA_TRY(flow_solve(k, M, NT.data(), NR.data(), R0.data(), blocks, p->probs.size(), &nodes, &pl->join,
                        &pl->cost));
  }
  pl->choice.resize(k);
  pl->dev.resize(k);
  for (size_t s2 = 0; s2 < k; ++s2) {
    pl->choice[s2] = nodes[s2] % (uint32_t)C;
    pl->dev[s2] = nodes[s2] >= C ? 1 : 0;
  }
  if (!pl->whole) {
    const LayoutDesc aos = layout_aos(p->shape);
    ADHA_TRY(place_plan(pl.get(), o->init == ADHA_INIT_AOS ? aos : pl->cands[pl->choice[0]]->d));
  }
  pl->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = pl.release();
  return result;
}

adha_status adha_plan_with_init(const adha_plan *src, adha_init init, adha_plan **out) {
  if (!src || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (enum_value(init) != ADHA_INIT_FREE && enum_value(init) != ADHA_INIT_AOS)
    return fail(ADHA_ERR_INVALID, "init must be FREE or AOS");
  if (src->hetero || !src->tokens.empty() || src->placed.empty())
    return fail(ADHA_ERR_UNSUPPORTED, "only linear GPU plans are solved again for another start");
  const size_t k = src->secs.size(), C = src->cands.size();
  if (src->T.size() != k * C || src->R.size() != C * C)
    return fail(ADHA_ERR_STATE, "the plan has no cost tables to solve again");
  std::unique_ptr<adha_plan> pl(new (std::nothrow) adha_plan);
  if (!pl) return fail(ADHA_ERR_OOM, "plan allocation failed");
  pl->shape = src->shape;
  pl->secs = src->secs;
  for (auto *l : src->cands) {
    adha_layout *c = new_layout(l->d);
    if (!c) return fail(ADHA_ERR_OOM, "layout allocation failed");
    pl->cands.push_back(c);
  }
  pl->T = src->T;
  pl->R = src->R;
  pl->whole = false;
  const LayoutDesc aos = layout_aos(src->shape);
  std::vector<double> R0(C, 0.0);
  if (init == ADHA_INIT_AOS)
    for (size_t c = 0; c < C; ++c)
      R0[c] = pl->cands[0]->d.same_groups(aos) ? pl->R[0 * C + c] : analytic_remap_us(aos, pl->cands[c]->d, false);
  ADHA_TRY(pdl_solve((uint32_t)k, (uint32_t)C, pl->T.data(), pl->R.data(), R0.data(), &pl->choice, &pl->cost));
  pl->dev.assign(k, 0);
  ADHA_TRY(place_plan(pl.get(), init == ADHA_INIT_AOS ? aos : pl->cands[pl->choice[0]]->d));
  pl->seconds = src->seconds;
  *out = pl.release();
  return ADHA_OK;
}

adha_status adha_plan_explicit(const adha_program *p, const adha_layout *const *layouts, const int32_t *devices,
                               adha_plan **out) {
  if (!p || !layouts || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  const size_t k = p->secs.size();
  std::unique_ptr<adha_plan> pl(new (std::nothrow) adha_plan);
  if (!pl) return fail(ADHA_ERR_OOM, "plan allocation failed");
  pl->shape = p->shape;
  pl->secs = p->secs;
  for (size_t s = 0; s < k; ++s) {
    if (!layouts[s] || !layouts[s]->d.shape.same(p->shape))
      return fail(ADHA_ERR_INVALID, "layout %zu is NULL or describes another struct", s);
    const int32_t d = devices ? devices[s] : 0;
    if (d != 0 && d != 1) return fail(ADHA_ERR_INVALID, "device %d of section %zu is not 0 (GPU) or 1 (host)", d, s);
    uint32_t c = 0;
    while (c < pl->cands.size() && !pl->cands[c]->d.same_map(layouts[s]->d)) ++c;
    if (c == pl->cands.size()) {
      adha_layout *l = new_layout(layouts[s]->d);
      if (!l) return fail(ADHA_ERR_OOM, "layout allocation failed");
      pl->cands.push_back(l);
    }
    pl->choice.push_back(c);
    pl->dev.push_back(d);
    pl->hetero |= d == 1;
  }
  const size_t C = pl->cands.size();
  pl->T.assign(k * C, 0.0);
  pl->R.assign(C * C, 0.0);
  if (pl->hetero) pl->TH.assign(k * C, 0.0);
  pl->tokens = p->tokens;
  pl->probs = p->probs;
  pl->join.assign(p->probs.size(), kNoJoin);
  pl->whole = !p->tokens.empty() || pl->hetero;
  if (!pl->whole && k) ADHA_TRY(place_plan(pl.get(), pl->cands[pl->choice[0]]->d));
  *out = pl.release();
  return ADHA_OK;
}

adha_status adha_plan_join(const adha_plan *pl, uint32_t i, uint32_t *candidate) {
  if (!pl || !candidate) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (i >= pl->join.size()) return fail(ADHA_ERR_INVALID, "branch %u out of range", i);
  if (pl->join[i] == kNoJoin) return fail(ADHA_ERR_STATE, "branch %u of an explicit plan has no join layout", i);
  *candidate = pl->join[i] % (uint32_t)pl->cands.size();
  return ADHA_OK;
}

adha_status adha_plan_device(const adha_plan *pl, uint32_t s, int32_t *device) {
  if (!pl || !device) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (s >= pl->choice.size()) return fail(ADHA_ERR_INVALID, "section %u out of range", s);
  *device = pl->dev.empty() ? 0 : pl->dev[s];
  return ADHA_OK;
}

adha_status adha_plan_nodes(const adha_plan *pl, uint32_t *M) {
  if (!pl || !M) return fail(ADHA_ERR_INVALID, "NULL argument");
  *M = (uint32_t)(pl->hetero ? 2 * pl->cands.size() : pl->cands.size());
  return ADHA_OK;
}

adha_status adha_plan_node_tables(const adha_plan *pl, double *T, double *R) {
  if (!pl) return fail(ADHA_ERR_INVALID, "NULL argument");
  std::vector<double> NT, NR;
  node_tables(pl, &NT, &NR);
  if (T) memcpy(T, NT.data(), NT.size() * sizeof(double));
  if (R) memcpy(R, NR.data(), NR.size() * sizeof(double));
  return ADHA_OK;
}

adha_status adha_plan_uniform(const adha_program *p, const adha_layout *l, adha_plan **out) {
  if (!p || !l || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!p->shape.same(l->d.shape)) return fail(ADHA_ERR_INVALID, "layout describes another struct");
  auto *pl = new (std::nothrow) adha_plan;
  if (!pl) return fail(ADHA_ERR_OOM, "plan allocation failed");
  pl->shape = p->shape;
  pl->secs = p->secs;
  adha_layout *c = new_layout(l->d);
  if (!c) {
    delete pl;
    return fail(ADHA_ERR_OOM, "layout allocation failed");
  }
  pl->cands.push_back(c);
  pl->choice.assign(p->secs.size(), 0);
  pl->dev.assign(p->secs.size(), 0);
  pl->tokens = p->tokens;
  pl->probs = p->probs;
  pl->join.assign(p->probs.size(), 0);
  pl->T.assign(p->secs.size(), 0.0);
  pl->R.assign(1, 0.0);
  pl->whole = !p->tokens.empty();
  if (!pl->whole) {
    const adha_status ps = place_plan(pl, l->d);
    if (ps < 0) {
      delete pl;
      return ps;
    }
  }
  *out = pl;
  return ADHA_OK;
}

adha_status adha_plan_destroy(adha_plan *pl) {
  delete pl;
  return ADHA_OK;
}

adha_status adha_plan_n_candidates(const adha_plan *pl, uint32_t *out) {
  if (!pl || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  *out = (uint32_t)pl->cands.size();
  return ADHA_OK;
}

adha_status adha_plan_candidate(const adha_plan *pl, uint32_t c, const adha_layout **out) {
  if (!pl || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (c >= pl->cands.size()) return fail(ADHA_ERR_INVALID, "candidate %u out of range", c);
  *out = pl->cands[c];
  return ADHA_OK;
}

adha_status adha_plan_choice(const adha_plan *pl, uint32_t s, uint32_t *candidate) {
  if (!pl || !candidate) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (s >= pl->choice.size()) return fail(ADHA_ERR_INVALID, "section %u out of range", s);
  *candidate = pl->choice[s];
  return ADHA_OK;
}

adha_status adha_plan_cost(const adha_plan *pl, double *us) {
  if (!pl || !us) return fail(ADHA_ERR_INVALID, "NULL argument");
  *us = pl->cost;
  return ADHA_OK;
}

adha_status adha_plan_tables(const adha_plan *pl, double *T, double *R) {
  if (!pl) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (T && !pl->T.empty()) memcpy(T, pl->T.data(), pl->T.size() * sizeof(double));
  if (R && !pl->R.empty()) memcpy(R, pl->R.data(), pl->R.size() * sizeof(double));
  return ADHA_OK;
}

adha_status adha_plan_time(const adha_plan *pl, double *seconds) {
  if (!pl || !seconds) return fail(ADHA_ERR_INVALID, "NULL argument");
  *seconds = pl->seconds;
  return ADHA_OK;
}

adha_status adha_plan_verified(const adha_plan *pl, uint32_t *entries) {
  if (!pl || !entries) return fail(ADHA_ERR_INVALID, "NULL argument");
  *entries = pl->verified;
  return ADHA_OK;
}

adha_status adha_run(adha_ctx *ctx, const adha_plan *pl, const adha_layout *in_layout, void *buf_a,
                     void *buf_b, uint64_t buf_cap, const int32_t *idx, uint64_t idx_count, void *stream,
                     const adha_layout **out_layout, int32_t *out_in_b) {
  if (!ctx || !pl || !in_layout || !out_layout || !out_in_b) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!in_layout->d.shape.same(pl->shape)) return fail(ADHA_ERR_INVALID, "input layout describes another struct");
  for (int32_t d : pl->dev)
    if (d != 0) return fail(ADHA_ERR_INVALID, "the plan maps sections to the host: run it with adha_run_hetero");
  if (!pl->tokens.empty()) return fail(ADHA_ERR_INVALID, "the program has branches: run it with adha_run_flow");
  // validate everything before the first launch
  const adha_layout *cur = in_layout;
  bool in_b = false, needs_b = false;
  uint64_t need = in_layout->d.nbytes;
  for (size_t s = 0; s < pl->secs.size(); ++s) {
    const adha_layout *L = pl->cands[pl->choice[s]];
    need = std::max(need, L->d.nbytes);
    if (!cur->d.same_map(L->d)) needs_b = true;
    cur = L;
    adha_section tmp;
    tmp.d = pl->secs[s];
    ADHA_TRY(validate_section_run(&tmp, L, buf_a, buf_cap, idx, idx_count));
  }
  if (buf_cap < need) return fail(ADHA_ERR_INVALID, "buffers hold %llu bytes, the plan needs %llu",
                                  (unsigned long long)buf_cap, (unsigned long long)need);
  if (need && (!buf_a || ((uintptr_t)buf_a & 255u))) return fail(ADHA_ERR_INVALID, "buf_a is NULL or misaligned");
  if (needs_b && need && (!buf_b || ((uintptr_t)buf_b & 255u)))
    return fail(ADHA_ERR_INVALID, "buf_b is NULL or misaligned and the plan remaps");
  if (needs_b && buf_b) {
    uintptr_t x = (uintptr_t)buf_a, y = (uintptr_t)buf_b;
    if (x < y + need && y < x + need) return fail(ADHA_ERR_INVALID, "buf_a and buf_b overlap");
  }
  for (const SectionDesc &d : pl->secs)
    if (d.op == ADHA_OP_REDUCE && need) {
      const uintptr_t o = (uintptr_t)d.out, no = (uintptr_t)d.reduce_cells() * 8;
      for (const void *b : {(const void *)buf_a, needs_b ? (const void *)buf_b : nullptr})
        if (b && o < (uintptr_t)b + need && (uintptr_t)b < o + no)
          return fail(ADHA_ERR_INVALID, "a reduction's result table overlaps the data buffers");
    }
  DeviceGuard g(ctx->c.device);
  hipStream_t st = (hipStream_t)stream;
  cur = in_layout;
  for (size_t s = 0; s < pl->secs.size(); ++s) {
    const adha_layout *L = pl->cands[pl->choice[s]];
    if (!cur->d.same_map(L->d)) {
      void *from = in_b ? buf_b : buf_a, *to = in_b ? buf_a : buf_b;
      ADHA_TRY(remap_one(&ctx->c, cur, from, L, to, st));
      in_b = !in_b;
      cur = L;
    }
    ADHA_TRY(section_launch(&ctx->c, pl->secs[s], L->d, in_b ? buf_b : buf_a, idx, st));
  }
  *out_layout = cur;
  *out_in_b = in_b ? 1 : 0;
  return ADHA_OK;
}

adha_status adha_plan_arena(const adha_plan *pl, uint64_t *bytes, const adha_layout **start,
                            const adha_layout **end) {
  if (!pl) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (pl->placed.empty())
    return fail(ADHA_ERR_UNSUPPORTED, "structured programs and plans over both devices do not run placed");
  if (bytes) *bytes = pl->arena;
  if (start) *start = pl->placed.front();
  if (end) *end = pl->placed.back();
  return ADHA_OK;
}

adha_status adha_plan_placed(const adha_plan *pl, uint32_t i, const adha_layout **out) {
  if (!pl || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (pl->placed.empty())
    return fail(ADHA_ERR_UNSUPPORTED, "structured programs and plans over both devices do not run placed");
  if (i >= pl->placed.size()) return fail(ADHA_ERR_INVALID, "index %u out of range", i);
  *out = pl->placed[i];
  return ADHA_OK;
}

adha_status adha_run_placed(adha_ctx *ctx, const adha_plan *pl, void *arena, uint64_t arena_cap,
                            const int32_t *idx, uint64_t idx_count, void *stream) {
  if (!ctx || !pl) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (pl->placed.empty())
    return fail(ADHA_ERR_UNSUPPORTED, "structured programs and plans over both devices do not run placed");
  for (int32_t d : pl->dev)
    if (d != 0) return fail(ADHA_ERR_INVALID, "the plan maps sections to the host: run it with adha_run_hetero");
  const uint64_t need = pl->arena;
  if (need && (!arena || ((uintptr_t)arena & 255u))) return fail(ADHA_ERR_INVALID, "arena is NULL or misaligned");
  if (arena_cap < need)
    return fail(ADHA_ERR_INVALID, "the arena holds %llu bytes, the plan needs %llu", (unsigned long long)arena_cap,
                (unsigned long long)need);
  // validate everything before the first launch
  for (size_t s = 0; s < pl->secs.size(); ++s) {
    adha_section tmp;
    tmp.d = pl->secs[s];
    ADHA_TRY(validate_section_run(&tmp, pl->placed[s + 1], arena, arena_cap, idx, idx_count));
    if (tmp.d.op == ADHA_OP_REDUCE && need) {
      const uintptr_t o = (uintptr_t)tmp.d.out, no = (uintptr_t)tmp.d.reduce_cells() * 8;
      if (o < (uintptr_t)arena + need && (uintptr_t)arena < o + no)
        return fail(ADHA_ERR_INVALID, "a reduction's result table overlaps the arena");
    }
  }
  DeviceGuard g(ctx->c.device);
  hipStream_t st = (hipStream_t)stream;
  const adha_layout *cur = pl->placed[0];
  for (size_t s = 0; s < pl->secs.size(); ++s) {
    const adha_layout *L = pl->placed[s + 1];
    if (!cur->d.same_map(L->d)) ADHA_TRY(remap_in_place(&ctx->c, cur->d, L->d, arena, st));
    ADHA_TRY(section_launch(&ctx->c, pl->secs[s], L->d, arena, idx, st));
    cur = L;
  }
  return ADHA_OK;
}

adha_status adha_run_hetero(adha_ctx *ctx, const adha_plan *pl, const adha_layout *in_layout, int32_t in_device,
                            void *dev_a, void *dev_b, void *host_a, void *host_b, uint64_t buf_cap,
                            const int32_t *idx_dev, const int32_t *idx_host, uint64_t idx_count, void *stream,
                            const adha_layout **out_layout, int32_t *out_device, int32_t *out_in_b) {
  if (!ctx || !pl || !in_layout || !out_layout || !out_device || !out_in_b)
    return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!in_layout->d.shape.same(pl->shape)) return fail(ADHA_ERR_INVALID, "input layout describes another struct");
  if (in_device != 0 && in_device != 1) return fail(ADHA_ERR_INVALID, "in_device must be 0 (GPU) or 1 (host)");
  if (!pl->tokens.empty()) return fail(ADHA_ERR_UNSUPPORTED, "programs with branches run on the GPU (adha_run_flow)");
  // validate everything before the first launch or copy
  const size_t k = pl->secs.size();
  uint64_t need = in_layout->d.nbytes;
  bool uses_host = in_device == 1, uses_dev = in_device == 0, host_gather = false, dev_gather = false;
  int at = in_device;
  for (size_t s = 0; s < k; ++s) {
    const adha_layout *L = pl->cands[pl->choice[s]];
    need = std::max(need, L->d.nbytes);
    const int d = pl->dev.empty() ? 0 : pl->dev[s];
    uses_host |= d == 1;
    uses_dev |= d == 0 || d != at;  // a move between devices goes through the GPU's buffers
    at = d;
    if (pl->secs[s].degree && !pl->secs[s].stencil) (d == 1 ? host_gather : dev_gather) = true;
  }
  const int64_t n = pl->shape.n;
  if (need) {
    if (buf_cap < need)
      return fail(ADHA_ERR_INVALID, "buffers hold %llu bytes, the plan needs %llu", (unsigned long long)buf_cap,
                  (unsigned long long)need);
    if (uses_dev && (!dev_a || !dev_b || ((uintptr_t)dev_a & 255u) || ((uintptr_t)dev_b & 255u)))
      return fail(ADHA_ERR_INVALID, "device buffers are NULL or misaligned");
    if (uses_host && (!host_a || !host_b)) return fail(ADHA_ERR_INVALID, "host buffers are NULL");
    const void *bufs[4] = {dev_a, dev_b, host_a, host_b};
    for (int x = 0; x < 4; ++x)
      for (int y = x + 1; y < 4; ++y)
        if (bufs[x] && bufs[y] && (uintptr_t)bufs[x] < (uintptr_t)bufs[y] + need &&
            (uintptr_t)bufs[y] < (uintptr_t)bufs[x] + need)
          return fail(ADHA_ERR_INVALID, "buffers overlap");
  }
  if (n > 0) {
    uint32_t maxd = 0;
    for (auto &d : pl->secs)
      if (!d.stencil) maxd = std::max(maxd, d.degree);
    if (host_gather && (!idx_host || idx_count < (uint64_t)n * maxd))
      return fail(ADHA_ERR_INVALID, "a gather on the host needs a host index array of N*d entries");
    if (dev_gather && (!idx_dev || ((uintptr_t)idx_dev & 255u) || idx_count < (uint64_t)n * maxd))
      return fail(ADHA_ERR_INVALID, "a gather on the GPU needs a device index array of N*d entries");
    for (const SectionDesc &d : pl->secs)
      if (d.op == ADHA_OP_REDUCE && need) {
        const uintptr_t o = (uintptr_t)d.out, no = (uintptr_t)d.reduce_cells() * 8;
        for (const void *b : {(const void *)dev_a, (const void *)dev_b})
          if (b && o < (uintptr_t)b + need && (uintptr_t)b < o + no)
            return fail(ADHA_ERR_INVALID, "a reduction's result table overlaps the data buffers");
      }
  }
  DeviceGuard g(ctx->c.device);
  hipStream_t st = (hipStream_t)stream;
  const uint32_t threads = host_threads(&ctx->c);
  void *bufs[2][2] = {{dev_a, dev_b}, {host_a, host_b}};
  int where = in_device, which = 0;
  const adha_layout *cur = in_layout;
  for (size_t s = 0; s < k; ++s) {
    const adha_layout *L = pl->cands[pl->choice[s]];
    const int dev = pl->dev.empty() ? 0 : pl->dev[s];
    const bool remap = !cur->d.same_map(L->d);
    if (dev == where) {
      if (remap) {
        if (where == 0) ADHA_TRY(remap_one(&ctx->c, cur, bufs[0][which], L, bufs[0][!which], st));
        else ADHA_TRY(host_remap(threads, cur->d, (const uint8_t *)bufs[1][which], L->d, (uint8_t *)bufs[1][!which]));
        which = !which;
      }
    } else if (where == 0) {  // GPU -> host: remap on the GPU first
      if (remap) {
        ADHA_TRY(remap_one(&ctx->c, cur, bufs[0][which], L, bufs[0][!which], st));
        which = !which;
      }
      ADHA_HIP(hipMemcpyAsync(bufs[1][which], bufs[0][which], L->d.nbytes, hipMemcpyDeviceToHost, st));
      ADHA_HIP(hipStreamSynchronize(st));
    } else {  // host -> GPU: copy, then remap on the GPU
      ADHA_HIP(hipMemcpyAsync(bufs[0][which], bufs[1][which], cur->d.nbytes, hipMemcpyHostToDevice, st));
      if (remap) {
        ADHA_TRY(remap_one(&ctx->c, cur, bufs[0][which], L, bufs[0][!which], st));
        which = !which;
      }
    }
    where = dev;
    cur = L;
    const SectionDesc &sec = pl->secs[s];
    if (dev == 0) {
      ADHA_TRY(section_launch(&ctx->c, sec, L->d, bufs[0][which], idx_dev, st));
    } else {
      ADHA_HIP(hipStreamSynchronize(st));
      std::vector<uint64_t> table(sec.op == ADHA_OP_REDUCE ? sec.reduce_cells() : 0);
      uint64_t bad = 0;
      ADHA_TRY(host_section_run(threads, sec, L->d, (uint8_t *)bufs[1][which], idx_host, table.data(), &bad));
      ctx->c.host_bad += bad;
      if (sec.op == ADHA_OP_REDUCE)
        ADHA_HIP(hipMemcpy(sec.out, table.data(), table.size() * 8, hipMemcpyHostToDevice));
    }
  }
  if (where == 1) ADHA_HIP(hipStreamSynchronize(st));
  *out_layout = cur;
  *out_device = where;
  *out_in_b = which;
  return ADHA_OK;
}

adha_status adha_run_flow(adha_ctx *ctx, const adha_plan *pl, const adha_layout *in_layout, void *buf_a,
                          void *buf_b, uint64_t buf_cap, const int32_t *idx, uint64_t idx_count,
                          const uint8_t *taken, uint32_t n_taken, void *stream, const adha_layout **out_layout,
                          int32_t *out_in_b) {
  if (!ctx || !pl || !in_layout || !out_layout || !out_in_b) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (!in_layout->d.shape.same(pl->shape)) return fail(ADHA_ERR_INVALID, "input layout describes another struct");
  for (int32_t d : pl->dev)
    if (d != 0) return fail(ADHA_ERR_UNSUPPORTED, "branches run GPU sections only");
  const size_t k = pl->secs.size();
  // the walk: the sequence of (section or join) steps along the outcomes
  std::vector<int32_t> tok = pl->tokens;
  if (tok.empty())
    for (size_t s2 = 0; s2 < k; ++s2) tok.push_back((int32_t)s2);
  size_t n_if = 0;
  for (int32_t x : tok) n_if += x == ADHA_TOK_IF;
  if (n_if && (!taken || n_taken < n_if)) return fail(ADHA_ERR_INVALID, "%zu branch outcomes are needed", n_if);
  struct Step {
    int sec;          // >= 0: run this section
    uint32_t join;    // else: move to this join candidate (kNoJoin: stay)
  };
  std::vector<FlowBlock> blocks;
  ADHA_TRY(parse_flow(tok, pl->probs, k, &blocks));
  std::vector<Step> steps;
  // the blocks along the outcomes: a branch runs the part taken, then moves
  // to its join layout
  std::vector<std::pair<int, int>> stack{{0, 0}};  // (block, next item)
  while (!stack.empty()) {
    auto &[id, pos] = stack.back();
    const FlowBlock &b = blocks[id];
    if (b.kind == 0) {
      steps.push_back({b.sec, 0});
      stack.pop_back();
    } else if (b.kind == 1) {
      if (pos < (int)b.items.size()) {
        const int c = b.items[pos++];
        stack.push_back({c, 0});
      } else {
        stack.pop_back();
      }
    } else {
      if (pos == 0) {
        pos = 1;
        stack.push_back({taken[b.branch] ? b.first : b.second, 0});
      } else {
        steps.push_back({-1, pl->join.empty() ? kNoJoin : pl->join[b.branch]});
        stack.pop_back();
      }
    }
  }
  uint64_t need = in_layout->d.nbytes;
  for (const Step &st2 : steps) {
    const adha_layout *L = st2.sec >= 0 ? pl->cands[pl->choice[st2.sec]]
                                        : (st2.join == kNoJoin ? nullptr : pl->cands[st2.join % pl->cands.size()]);
    if (!L) continue;
    need = std::max(need, L->d.nbytes);
    if (st2.sec >= 0) {
      adha_section tmp;
      tmp.d = pl->secs[st2.sec];
      ADHA_TRY(validate_section_run(&tmp, L, buf_a, buf_cap, idx, idx_count));
    }
  }
  if (buf_cap < need) return fail(ADHA_ERR_INVALID, "buffers hold %llu bytes, the plan needs %llu",
                                  (unsigned long long)buf_cap, (unsigned long long)need);
  if (need && (!buf_a || !buf_b || ((uintptr_t)buf_a & 255u) || ((uintptr_t)buf_b & 255u)))
    return fail(ADHA_ERR_INVALID, "buffers are NULL or misaligned");
  {
    const uintptr_t x = (uintptr_t)buf_a, y = (uintptr_t)buf_b;
    if (need && x < y + need && y < x + need) return fail(ADHA_ERR_INVALID, "buf_a and buf_b overlap");
  }
  DeviceGuard g(ctx->c.device);
  hipStream_t st = (hipStream_t)stream;
  const adha_layout *cur = in_layout;
  bool in_b = false;
  for (const Step &st2 : steps) {
    const adha_layout *L = st2.sec >= 0 ? pl->cands[pl->choice[st2.sec]]
                                        : (st2.join == kNoJoin ? nullptr : pl->cands[st2.join % pl->cands.size()]);
    if (!L) continue;
    if (!cur->d.same_map(L->d)) {
      ADHA_TRY(remap_one(&ctx->c, cur, in_b ? buf_b : buf_a, L, in_b ? buf_a : buf_b, st));
      in_b = !in_b;
    }
    cur = L;
    if (st2.sec >= 0) ADHA_TRY(section_launch(&ctx->c, pl->secs[st2.sec], L->d, in_b ? buf_b : buf_a, idx, st));
  }
  *out_layout = cur;
  *out_in_b = in_b ? 1 : 0;
  return ADHA_OK;
}

}  // extern "C"
