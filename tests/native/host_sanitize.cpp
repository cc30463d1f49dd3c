// Host-side checks built with the compiler's sanitizers (AddressSanitizer
// with UndefinedBehaviorSanitizer, or ThreadSanitizer) by
// tests/test_host_sanitizers.py.  No GPU work: struct, layout and section
// handles, the greedy grouping and the analytic planner, placed layouts,
// the remap descriptor check, the host backend's sections and remaps (many
// small jobs through its thread pool), argument errors, the trainer's
// scratch-size check, and the oracle's C routines.  Every host result is
// also checked: sections give the same record values under every layout,
// and remaps are inverted exactly.
//
//   host_sanitize all   -- everything (ASan/UBSan build)
//   host_sanitize pool  -- the thread-pool stress alone (TSan build)
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "adha.h"
#include "adha_impl.h"

extern "C" {
uint64_t orc_layout_addr(const uint64_t *desc, int32_t f, int64_t r);
void orc_remap(int32_t n_fields, const uint64_t *src_desc, const uint8_t *src, const uint64_t *dst_desc,
               uint8_t *dst, int64_t r_begin, int64_t r_end);
int64_t orc_section(int32_t op, int64_t n, const uint64_t *desc, const int32_t *dtypes, int32_t n_read,
                    const int32_t *rd, int32_t n_write, const int32_t *wr, int32_t degree, const int32_t *idx,
                    uint8_t *buf, int64_t r_begin, int64_t r_end);
}

namespace {

int g_failures = 0;

#define CHECK(cond)                                                             \
  do {                                                                          \
    if (!(cond)) {                                                              \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond);   \
      ++g_failures;                                                             \
    }                                                                           \
  } while (0)
#define OK(call) CHECK((call) >= 0)
#define FAILS(call) CHECK((call) < 0)

// SplitMix64: the seeded values of the checks.
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  uint32_t below(uint32_t n) { return (uint32_t)(((next() >> 32) * n) >> 32); }
};

// 32 fields: 20 F32, 8 I32, 4 F64 (the multi-section workload's record).
adha_struct *make_struct(int64_t n) {
  adha_struct *s = nullptr;
  OK(adha_struct_create(n, &s));
  for (int f = 0; f < 32; ++f) {
    int32_t id = -1;
    const adha_dtype dt = f < 20 ? ADHA_F32 : f < 28 ? ADHA_I32 : ADHA_F64;
    OK(adha_struct_add_field(s, dt, dt == ADHA_F64 ? 8 : 4, &id));
    CHECK(id == f);
  }
  return s;
}

// Record values: finite floats for F32/F64 fields, any bits for I32.
void fill_aos(const adha_layout *aos, int64_t n, std::vector<uint8_t> &buf, Rng &g) {
  uint64_t nb = 0;
  OK(adha_layout_nbytes(aos, &nb));
  buf.assign(nb, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int f = 0; f < 32; ++f) {
      uint64_t at = 0;
      OK(adha_layout_addr(aos, r, f, &at));
      if (f < 20) {
        const float v = (float)((int32_t)g.below(2000001) - 1000000) / 65536.0f;
        std::memcpy(&buf[at], &v, 4);
      } else if (f < 28) {
        const uint32_t v = (uint32_t)g.next();
        std::memcpy(&buf[at], &v, 4);
      } else {
        const double v = (double)((int64_t)g.below(2000001) - 1000000) / 4096.0;
        std::memcpy(&buf[at], &v, 8);
      }
    }
}

adha_layout *random_layout(const adha_struct *s, Rng &g) {
  uint32_t gof[32], tiles[32];
  const uint32_t ng = 1 + g.below(8);
  for (int f = 0; f < 32; ++f) gof[f] = f < (int)ng ? (uint32_t)f : g.below(ng);
  for (uint32_t k = 0; k < ng; ++k) tiles[k] = 1u << g.below(9);
  adha_layout *l = nullptr;
  OK(adha_layout_create(s, ng, gof, tiles, &l));
  return l;
}

std::vector<adha_section *> random_sections(const adha_struct *s, Rng &g, int k) {
  std::vector<adha_section *> out;
  for (int i = 0; i < k; ++i) {
    int32_t perm[32];
    for (int f = 0; f < 32; ++f) perm[f] = f;
    for (int f = 31; f > 0; --f) std::swap(perm[f], perm[g.below(f + 1)]);
    const uint32_t nr = 2 + g.below(9), nw = 1 + g.below(2);
    const uint32_t d = g.below(2) ? 0 : 1 + g.below(16);
    adha_section *sec = nullptr;
    OK(adha_section_create(s, ADHA_OP_GEN, nr, perm, nw, perm + nr, d, &sec));
    out.push_back(sec);
  }
  return out;
}

// Sections on the host backend under several layouts give the same record
// values (read back through a remap to AoS).
void check_host_sections(int64_t n, uint32_t threads) {
  Rng g{11 + (uint64_t)n};
  adha_struct *s = make_struct(n);
  adha_layout *aos = nullptr, *soa = nullptr;
  OK(adha_layout_aos(s, &aos));
  OK(adha_layout_soa(s, &soa));
  std::vector<uint8_t> src;
  fill_aos(aos, n, src, g);
  std::vector<int32_t> idx((size_t)n * 16);
  for (auto &v : idx) v = (int32_t)g.below((uint32_t)n);
  std::vector<adha_section *> secs = random_sections(s, g, 8);
  std::vector<adha_layout *> lays{aos, soa};
  for (int i = 0; i < 4; ++i) lays.push_back(random_layout(s, g));
  std::vector<uint8_t> ref;
  for (adha_layout *l : lays) {
    uint64_t nb = 0, na = 0;
    OK(adha_layout_nbytes(l, &nb));
    OK(adha_layout_nbytes(aos, &na));
    std::vector<uint8_t> buf(nb), back(na);
    OK(adha_host_remap(aos, src.data(), src.size(), l, buf.data(), buf.size(), threads));
    for (adha_section *sec : secs) {
      uint64_t bad = 0;
      OK(adha_host_section_run(sec, l, buf.data(), buf.size(), idx.data(), idx.size(), nullptr, 0, threads, &bad));
      CHECK(bad == 0);
    }
    OK(adha_host_remap(l, buf.data(), buf.size(), aos, back.data(), back.size(), threads));
    if (ref.empty()) ref = back;
    else CHECK(ref == back);
  }
  // a reduction over F32 and F64 fields keyed by an I32 field (values in [0, 5))
  {
    std::vector<uint8_t> buf = src;
    for (int64_t r = 0; r < n; ++r) {
      uint64_t at = 0;
      OK(adha_layout_addr(aos, r, 24, &at));
      const int32_t k = (int32_t)g.below(5);
      std::memcpy(&buf[at], &k, 4);
    }
    const int32_t rd[4] = {0, 3, 17, 29};
    // the section's own result array must be 256-byte aligned (a device
    // array in GPU runs); host runs write the table they are given
    std::vector<uint64_t> store(5 * 5 + 32);
    uint64_t *dev_like = reinterpret_cast<uint64_t *>((reinterpret_cast<uintptr_t>(store.data()) + 255) & ~uintptr_t(255));
    std::vector<uint64_t> t1(5 * 5), t2(5 * 5);
    adha_section *red = nullptr;
    OK(adha_section_create_reduce(s, 4, rd, 24, 5, dev_like, 25 * 8, &red));
    uint64_t bad = 0;
    OK(adha_host_section_run(red, aos, buf.data(), buf.size(), nullptr, 0, t1.data(), t1.size() * 8, threads, &bad));
    CHECK(bad == 0);
    // the same under SoA: the same bits (fixed order, compensated)
    uint64_t nb = 0;
    OK(adha_layout_nbytes(soa, &nb));
    std::vector<uint8_t> sbuf(nb);
    OK(adha_host_remap(aos, buf.data(), buf.size(), soa, sbuf.data(), sbuf.size(), threads));
    OK(adha_host_section_run(red, soa, sbuf.data(), sbuf.size(), nullptr, 0, t2.data(), t2.size() * 8, threads, &bad));
    CHECK(t1 == t2);
    uint64_t count = 0;
    for (int k = 0; k < 5; ++k) count += t1[k * 5 + 4];
    CHECK(count == (uint64_t)n);
    // a table too small for the reduction is refused
    FAILS(adha_host_section_run(red, aos, buf.data(), buf.size(), nullptr, 0, t1.data(), 8, threads, &bad));
    OK(adha_section_destroy(red));
  }
  for (adha_section *sec : secs) OK(adha_section_destroy(sec));
  for (adha_layout *l : lays) OK(adha_layout_destroy(l));
  OK(adha_struct_destroy(s));
}

// The analytic planner (no device), placed layouts, flows and the solvers.
void check_planner() {
  Rng g{5};
  const int64_t n = 1 << 16;
  adha_struct *s = make_struct(n);
  std::vector<adha_section *> secs = random_sections(s, g, 8);
  adha_program *p = nullptr;
  OK(adha_program_create(s, (uint32_t)secs.size(), secs.data(), &p));
  std::vector<uint64_t> w(32 * 32);
  OK(adha_affinity(p, 0, 7, w.data()));
  for (uint32_t cap : {16u, 64u, 128u, 4096u}) {
    adha_layout *l = nullptr;
    OK(adha_ods(p, 0, 7, cap, 1, &l));
    OK(adha_layout_destroy(l));
  }
  FAILS(adha_ods(p, 3, 2, 64, 1, nullptr));
  adha_plan_opts o;
  OK(adha_plan_opts_default(&o));
  o.cost = ADHA_COST_ANALYTIC;
  o.catalogue = ADHA_CAT_FULL;
  adha_plan *pl = nullptr;
  OK(adha_plan_create(nullptr, p, &o, nullptr, 0, nullptr, &pl));
  uint32_t C = 0;
  OK(adha_plan_n_candidates(pl, &C));
  CHECK(C >= 3);
  std::vector<double> T(8 * C), R((size_t)C * C);
  OK(adha_plan_tables(pl, T.data(), R.data()));
  std::vector<uint32_t> path(8);
  double cost = 0.0, pc = 0.0;
  OK(adha_pdl_solve(8, C, T.data(), R.data(), nullptr, path.data(), &cost));
  OK(adha_plan_cost(pl, &pc));
  CHECK(cost == pc);
  for (uint32_t i = 0; i < 8; ++i) {
    uint32_t c = 0;
    OK(adha_plan_choice(pl, i, &c));
    CHECK(c == path[i]);
  }
  uint64_t arena = 0;
  const adha_layout *start = nullptr, *end = nullptr;
  OK(adha_plan_arena(pl, &arena, &start, &end));
  for (uint32_t i = 0; i <= 8; ++i) {  // the start layout, then one per section
    const adha_layout *pli = nullptr;
    OK(adha_plan_placed(pl, i, &pli));
    uint64_t nb = 0;
    OK(adha_layout_nbytes(pli, &nb));
    CHECK(nb <= arena);
  }
  FAILS(adha_plan_placed(pl, 9, &start));
  adha_plan *fixed = nullptr;
  OK(adha_plan_with_init(pl, ADHA_INIT_AOS, &fixed));
  OK(adha_plan_destroy(fixed));
  // remap descriptors of candidate pairs (checked on the host)
  for (uint32_t a = 0; a < C; a += 3)
    for (uint32_t b = 0; b < C; b += 5) {
      const adha_layout *la = nullptr, *lb = nullptr;
      OK(adha_plan_candidate(pl, a, &la));
      OK(adha_plan_candidate(pl, b, &lb));
      adha_remap_info info;
      OK(adha_remap_describe(la, lb, 256, &info));
    }
  OK(adha_plan_destroy(pl));
  // a structured program: the expected-cost path over its branches
  const int32_t tok[] = {0, 1, ADHA_TOK_IF, 2, 3, ADHA_TOK_ELSE, 4, ADHA_TOK_END, 5, ADHA_TOK_IF, 6, ADHA_TOK_END, 7};
  const double probs[] = {0.6, 0.3};
  OK(adha_program_set_flow(p, 13, tok, probs));
  OK(adha_plan_create(nullptr, p, &o, nullptr, 0, nullptr, &pl));
  OK(adha_plan_tables(pl, T.data(), R.data()));
  uint32_t node[8], join[2], st = 0;
  OK(adha_flow_solve(8, C, T.data(), R.data(), nullptr, 13, tok, probs, node, join, &st, &cost));
  OK(adha_plan_destroy(pl));
  const int32_t bad_tok[] = {0, ADHA_TOK_IF, 1, ADHA_TOK_ELSE, 2};  // unclosed branch
  FAILS(adha_program_set_flow(p, 5, bad_tok, probs));
  OK(adha_program_destroy(p));
  // placed layouts: disjoint regions are accepted, overlapping ones refused
  adha_layout *soa = nullptr, *pls = nullptr;
  OK(adha_layout_soa(s, &soa));
  std::vector<uint64_t> bases(32);
  OK(adha_layout_bases(soa, bases.data()));
  uint64_t total = 0;
  OK(adha_layout_nbytes(soa, &total));
  // the groups in reverse order, each right after the next one's region
  std::vector<uint64_t> size(32), rev(32);
  for (int gi = 0; gi < 32; ++gi) size[gi] = (gi < 31 ? bases[gi + 1] : total) - bases[gi];
  uint64_t at = 0;
  for (int gi = 31; gi >= 0; --gi) {
    rev[gi] = at;
    at += size[gi];
  }
  OK(adha_layout_place(soa, 32, rev.data(), &pls));
  uint64_t placed_bytes = 0;
  OK(adha_layout_nbytes(pls, &placed_bytes));
  CHECK(placed_bytes == total);
  OK(adha_layout_destroy(pls));
  rev[1] = rev[0];
  FAILS(adha_layout_place(soa, 32, rev.data(), &pls));
  rev[1] = 100;  // not a multiple of 256
  FAILS(adha_layout_place(soa, 32, rev.data(), &pls));
  OK(adha_layout_destroy(soa));
  for (adha_section *sec : secs) OK(adha_section_destroy(sec));
  OK(adha_struct_destroy(s));
}

void check_argument_errors() {
  adha_struct *s = nullptr;
  FAILS(adha_struct_create(-1, &s));
  FAILS(adha_struct_create(10, nullptr));
  OK(adha_struct_create(10, &s));
  int32_t id = 0;
  FAILS(adha_struct_add_field(s, ADHA_F32, 8, &id));
  FAILS(adha_struct_add_field(s, ADHA_U16, 4, &id));
  FAILS(adha_struct_add_field(s, (adha_dtype)99, 4, &id));
  OK(adha_struct_add_field(s, ADHA_F32, 4, &id));
  OK(adha_struct_add_field(s, ADHA_U8, 1, &id));
  OK(adha_struct_add_field(s, ADHA_I16, 2, &id));
  adha_section *sec = nullptr;
  const int32_t rd[2] = {0, 1}, wr[1] = {2}, bad[1] = {7};
  FAILS(adha_section_create(s, ADHA_OP_GEN, 2, rd, 1, bad, 0, &sec));
  FAILS(adha_section_create(s, ADHA_OP_GEN, 2, rd, 1, rd, 3, &sec));  // a gather writing what it reads
  FAILS(adha_section_create(s, ADHA_OP_SUM, 2, rd, 1, wr, 0, &sec));  // SUM into an integer field
  OK(adha_section_create(s, ADHA_OP_GEN, 2, rd, 1, wr, 0, &sec));
  adha_layout *l = nullptr;
  const uint32_t gof[3] = {0, 0, 2}, tiles[3] = {1, 1, 1};
  FAILS(adha_layout_create(s, 3, gof, tiles, &l));  // label 1 unused
  const uint32_t gof2[3] = {0, 0, 1}, tiles2[2] = {3, 1};
  FAILS(adha_layout_create(s, 2, gof2, tiles2, &l));  // tile not a power of two
  uint64_t addr = 0;
  OK(adha_layout_aos(s, &l));
  FAILS(adha_layout_addr(l, 10, 0, &addr));
  FAILS(adha_layout_addr(l, 0, 3, &addr));
  std::vector<uint8_t> buf(64);
  uint64_t badc = 0;
  FAILS(adha_host_section_run(sec, l, buf.data(), 8, nullptr, 0, nullptr, 0, 2, &badc));  // buffer too small
  CHECK(adha_last_error() != nullptr && std::strlen(adha_last_error()) > 0);
  OK(adha_layout_destroy(l));
  OK(adha_section_destroy(sec));
  OK(adha_struct_destroy(s));
  OK(adha_struct_destroy(nullptr));  // like free(NULL)
}

// The trainer's backward pass refuses scratch smaller than its batch needs
// before any launch.
void check_trainer_scratch() {
  const size_t need = adha::mlp_scratch_floats(64);
  CHECK(need > 0);
  CHECK(adha::mlp_backward(nullptr, nullptr, nullptr, nullptr, 64, nullptr, nullptr, nullptr, need - 1, nullptr) ==
        ADHA_ERR_INVALID);
  CHECK(adha::mlp_backward(nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, need, nullptr) ==
        ADHA_ERR_INVALID);
  CHECK(adha::mlp_scratch_floats(128) == 2 * need);
}

// Many small jobs back to back through the host backend's thread pool.
void check_pool(int rounds) {
  Rng g{3};
  const int64_t n = 97;
  adha_struct *s = make_struct(n);
  adha_layout *aos = nullptr, *soa = nullptr;
  OK(adha_layout_aos(s, &aos));
  OK(adha_layout_soa(s, &soa));
  std::vector<uint8_t> a, b;
  fill_aos(aos, n, a, g);
  uint64_t ns = 0;
  OK(adha_layout_nbytes(soa, &ns));
  b.assign(ns, 0);
  std::vector<adha_section *> secs = random_sections(s, g, 4);
  std::vector<int32_t> idx((size_t)n * 16);
  for (auto &v : idx) v = (int32_t)g.below((uint32_t)n);
  for (int r = 0; r < rounds; ++r) {
    const uint32_t threads = 1 + (uint32_t)(r % 8);
    uint64_t bad = 0;
    OK(adha_host_section_run(secs[r % secs.size()], aos, a.data(), a.size(), idx.data(), idx.size(), nullptr, 0,
                             threads, &bad));
    if (r % 16 == 0) {
      OK(adha_host_remap(aos, a.data(), a.size(), soa, b.data(), b.size(), threads));
      std::vector<uint8_t> back(a.size());
      OK(adha_host_remap(soa, b.data(), b.size(), aos, back.data(), back.size(), 8));
      CHECK(back == a);
    }
  }
  for (adha_section *sec : secs) OK(adha_section_destroy(sec));
  OK(adha_layout_destroy(aos));
  OK(adha_layout_destroy(soa));
  OK(adha_struct_destroy(s));
}

// The oracle's C routines on a small struct: remap there and back, and a
// section (its gather skips out-of-range indices and counts them).
void check_oracle() {
  const int F = 3;
  const int64_t n = 50;
  const uint64_t e[F] = {4, 8, 4};
  // AoS: one group of 16-byte records; SoA: three arrays
  uint64_t aos[F * 5], soa[F * 5];
  uint64_t p = 0, base = 0;
  for (int f = 0; f < F; ++f) {
    const uint64_t ra[5] = {0, 1, 16, p, e[f]};
    std::memcpy(aos + 5 * f, ra, sizeof ra);
    p += e[f];
    const uint64_t rs[5] = {base, 1, e[f], 0, e[f]};
    std::memcpy(soa + 5 * f, rs, sizeof rs);
    base += (n * e[f] + 255) / 256 * 256;
  }
  std::vector<uint8_t> src(16 * n), mid(base), back(16 * n, 0);
  Rng g{9};
  for (int64_t r = 0; r < n; ++r) {
    const float x = (float)g.below(1000);
    const double y = (double)g.below(1000);
    const int32_t z = (int32_t)g.next();
    std::memcpy(&src[16 * r], &x, 4);
    std::memcpy(&src[16 * r + 4], &y, 8);
    std::memcpy(&src[16 * r + 12], &z, 4);
  }
  orc_remap(F, aos, src.data(), soa, mid.data(), 0, n);
  orc_remap(F, soa, mid.data(), aos, back.data(), 0, n);
  CHECK(back == src);
  CHECK(orc_layout_addr(soa, 2, 3) == soa[10] + 12);
  const int32_t dts[F] = {ADHA_F32, ADHA_F64, ADHA_I32};
  const int32_t rd[2] = {0, 1}, wr[1] = {2};
  std::vector<int32_t> idx((size_t)n * 3);
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i % 7 == 0 ? -1 : (int32_t)(i % n);
  const int64_t bad = orc_section(ADHA_OP_GEN, n, soa, dts, 2, rd, 1, wr, 3, idx.data(), mid.data(), 0, n);
  int64_t want = 0;
  for (size_t i = 0; i < idx.size(); ++i) want += idx[i] < 0;
  CHECK(bad == want);
}

}  // namespace

int main(int argc, char **argv) {
  const bool pool_only = argc > 1 && std::strcmp(argv[1], "pool") == 0;
  if (pool_only) {
    check_pool(1500);
  } else {
    check_argument_errors();
    check_trainer_scratch();
    check_oracle();
    check_planner();
    check_host_sections(1, 3);
    check_host_sections(3001, 1);
    check_host_sections(3001, 8);
    check_pool(400);
  }
  if (g_failures) {
    std::fprintf(stderr, "%d checks failed\n", g_failures);
    return 1;
  }
  std::printf("host checks passed (%s)\n", pool_only ? "pool" : "all");
  return 0;
}
