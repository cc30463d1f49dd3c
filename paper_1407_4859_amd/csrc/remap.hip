// Layout remap kernels for CDNA4 (gfx950).
//
// A remap (section 2's remap edge; section 3's remap between the Medical
// program's CPU and GPU sections) rewrites a record array from one layout
// into another.  It does no arithmetic, so it is bound by HBM bandwidth; the
// design goal is that both the reads and the writes are long runs of
// 16-byte accesses whatever the two layouts are.
//
// Tiles.  Records are cut into tiles of R records, R a multiple of 64 and of
// every group tile T in both layouts.  Inside one tile every group of a
// layout then occupies one contiguous run of R*S_g bytes, so the tile's
// source is a handful of contiguous runs and so is its destination.
//
// Main kernel (persistent, one work list for one or many arrays).  Each
// 256-thread workgroup owns a contiguous range of tiles.  Per tile it
//   1. loads the source runs with 16-byte loads (thread t takes chunks
//      t, t+256, ...) and writes them into LDS, one padding dword every
//      2^shift dwords so that the transposing reads below spread over banks;
//   2. builds every 16-byte destination chunk from four LDS dwords and
//      stores it with one 16-byte store.
// The LDS position each destination dword comes from depends only on its
// place in the tile, so each thread computes its positions once per array
// and keeps them in registers; the per-tile work is loads, LDS traffic and
// stores only.  The next tile's loads are issued before the current tile's
// stores (software pipelining).
//
// Byte mode.  With 1- or 2-byte fields a destination dword can hold bytes of
// up to four different (record, field) elements, so step 2 assembles each
// destination dword from four LDS bytes instead of one LDS dword.  Each
// thread keeps the sixteen LDS byte positions of each of its chunks packed
// two to a register (LDS addresses fit in 16 bits); the loads, the LDS
// image of the source runs and the 16-byte stores are those of the dword
// mode.
//
// Tail kernel.  Records past the last full tile, the padding records of
// tiled groups and the gaps between groups are written by a simple
// per-dword kernel that decodes each destination byte on its own (through
// a per-byte field table when fields are narrower than a dword).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "adha_impl.h"

namespace adha {

struct RGroup {
  uint64_t base;   // byte offset of the group in its buffer
  uint64_t end;    // start of the next group, or the layout size
  uint64_t bytes;  // roundup(N, T) * S
  uint32_t S;      // group record bytes
  uint32_t logT;
  uint32_t tile_off;  // byte offset of the group's R-record run in the tile image
  uint32_t word_off;  // first entry of this group in word_field
  uint32_t byte_off;  // first entry of this group in byte_field
};

struct RField {
  uint32_t sg, dg;  // source / destination group
  uint32_t sp, dp;  // byte offset inside the group record
  uint32_t e;       // element bytes
  uint32_t pad;
};

struct RArray {
  const uint8_t *src;
  uint8_t *dst;
  int64_t n;
  uint64_t n_full;      // full tiles handled by the main kernel
  uint64_t tile_begin;  // global index of this array's first tile
  uint32_t R;           // records per tile
  uint32_t n_chunks;    // 16-byte chunks per tile
  uint32_t nsg, ndg, nf;
  uint32_t dword;  // every field is 4 or 8 bytes (word_field is filled)
  const RGroup *sgrp;
  const RGroup *dgrp;
  const RField *fld;
  const uint8_t *word_field;  // per destination group, the field of each record dword
  const uint8_t *byte_field;  // per destination group, the field of each record byte
};

struct RTail {
  uint32_t array, dgroup;
  uint64_t start, end;    // byte range of dst to fill
  uint64_t block_begin;   // first tail block of this region
};

constexpr int kBlock = 256;
constexpr uint32_t kTailDwordsPerBlock = 1024;

// ------------------------------------------------------------------ kernels
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ u32x4 load16(const uint8_t *p) {
  const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
  if constexpr (NT) return __builtin_nontemporal_load(q);
  else return *q;
}

template <bool NT>
__device__ __forceinline__ void store16(uint8_t *p, u32x4 v) {
  u32x4 *q = reinterpret_cast<u32x4 *>(p);
  if constexpr (NT) __builtin_nontemporal_store(v, q);
  else *q = v;
}

// K: 16-byte slots per thread; NT: streaming (non-temporal) global accesses;
// BY: byte mode (destination dwords assembled from LDS bytes).
// Workgroup w takes tiles w*tiles_per_wg .. +tiles_per_wg (contiguous) or,
// when `strided`, tiles w, w + G, w + 2G, ... so that at any moment the
// grid works on neighbouring tiles.
template <int K, bool NT, bool BY>
__global__ __launch_bounds__(kBlock) void remap_tiles_kernel(const RArray *__restrict__ arrays,
                                                             uint32_t n_arrays, uint64_t total_tiles,
                                                             uint64_t tiles_per_wg, uint32_t shift,
                                                             uint32_t strided,
                                                             const uint8_t *src_override,
                                                             uint8_t *dst_override) {
  extern __shared__ uint32_t lds[];
  const uint32_t t = threadIdx.x;
  uint64_t g, g_end, step;
  if (strided) {
    g = blockIdx.x;
    step = gridDim.x;
    g_end = total_tiles;
  } else {
    g = (uint64_t)blockIdx.x * tiles_per_wg;
    step = 1;
    g_end = min(total_tiles, g + tiles_per_wg);
  }
  if (g >= g_end) return;

  // array holding tile g (arrays sorted by tile_begin, each with >= 1 tile)
  uint32_t lo = 0, hi = n_arrays;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (arrays[mid].tile_begin <= g) lo = mid; else hi = mid;
  }
  uint32_t a = lo;

  while (g < g_end) {
    while (a + 1 < n_arrays && arrays[a + 1].tile_begin <= g) ++a;
    const RArray &A = arrays[a];
    const uint64_t stop = min(g_end, A.tile_begin + A.n_full);
    const uint32_t nsg = A.nsg, ndg = A.ndg;

    constexpr int P = BY ? 8 : 4;  // position registers per slot
    uint64_t ld_off[K], st_off[K];
    uint32_t ld_S[K], st_S[K], ld_pos[K];
    uint32_t st_pos[K][P];
    bool act[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t c = t + kBlock * k;
      act[k] = c < A.n_chunks;
      ld_off[k] = st_off[k] = 0;
      ld_S[k] = st_S[k] = ld_pos[k] = 0;
#pragma unroll
      for (int q = 0; q < P; ++q) st_pos[k][q] = 0;
      if (!act[k]) continue;
      const uint32_t o = 16u * c;
      uint32_t gs = 0;
      for (uint32_t i = 1; i < nsg; ++i)
        if (A.sgrp[i].tile_off <= o) gs = i;
      ld_off[k] = A.sgrp[gs].base + (o - A.sgrp[gs].tile_off);
      ld_S[k] = A.sgrp[gs].S;
      const uint32_t lp = 4u * c;
      ld_pos[k] = lp + (lp >> shift);
      uint32_t gd = 0;
      for (uint32_t i = 1; i < ndg; ++i)
        if (A.dgrp[i].tile_off <= o) gd = i;
      const RGroup D = A.dgrp[gd];
      st_off[k] = D.base + (o - D.tile_off);
      st_S[k] = D.S;
      if constexpr (BY) {
        // LDS byte address of each of the chunk's 16 destination bytes
        const uint32_t Td = 1u << D.logT, tileB = Td * D.S;
#pragma unroll
        for (uint32_t j = 0; j < 16; ++j) {
          const uint32_t ob = o - D.tile_off + j;
          const uint32_t qq = ob / tileB;
          const uint32_t within = ob - qq * tileB;
          const RField F = A.fld[A.byte_field[D.byte_off + (within >> D.logT)]];
          const uint32_t local = within - F.dp * Td;
          const uint32_t rin = local / F.e;
          const uint32_t eb = local - rin * F.e;
          const uint32_t rec = qq * Td + rin;
          const RGroup Sg = A.sgrp[F.sg];
          const uint32_t Ts = 1u << Sg.logT;
          const uint32_t pos = Sg.tile_off + (rec >> Sg.logT) * Ts * Sg.S + F.sp * Ts +
                               (rec & (Ts - 1)) * F.e + eb;
          const uint32_t w = pos >> 2;
          const uint32_t lb = 4u * (w + (w >> shift)) + (pos & 3u);
          st_pos[k][j >> 1] |= lb << (16u * (j & 1u));
        }
        continue;
      }
      const uint32_t Td = 1u << D.logT, Swd = D.S >> 2, tileW = Td * Swd;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t w = ((o - D.tile_off) >> 2) + q;
        const uint32_t qq = w / tileW;
        const uint32_t within = w - qq * tileW;
        const uint32_t col = within >> D.logT;
        const RField F = A.fld[A.word_field[D.word_off + col]];
        const uint32_t ew = F.e >> 2;
        const uint32_t local = within - (F.dp >> 2) * Td;
        const uint32_t rin = ew == 2 ? (local >> 1) : local;
        const uint32_t jj = local - rin * ew;
        const uint32_t rec = qq * Td + rin;
        const RGroup Sg = A.sgrp[F.sg];
        const uint32_t Ts = 1u << Sg.logT;
        const uint32_t pos = (Sg.tile_off >> 2) + (rec >> Sg.logT) * Ts * (Sg.S >> 2) +
                             (F.sp >> 2) * Ts + (rec & (Ts - 1)) * ew + jj;
        st_pos[k][q] = pos + (pos >> shift);
      }
    }

    const uint8_t *src = src_override ? src_override : A.src;
    uint8_t *dst = dst_override ? dst_override : A.dst;
    const uint64_t r_step = step * (uint64_t)A.R;
    uint64_t r0 = (g - A.tile_begin) * (uint64_t)A.R;
    u32x4 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (act[k]) v[k] = load16<NT>(src + ld_off[k] + r0 * ld_S[k]);

    while (g < stop) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (act[k]) {
          uint32_t *p = lds + ld_pos[k];
          p[0] = v[k].x;
          p[1] = v[k].y;
          p[2] = v[k].z;
          p[3] = v[k].w;
        }
      __syncthreads();
      const uint64_t cur = r0;
      g += step;
      if (g < stop) {
        r0 += r_step;
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (act[k]) v[k] = load16<NT>(src + ld_off[k] + r0 * ld_S[k]);
      }
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (act[k]) {
          u32x4 o;
          if constexpr (BY) {
            const uint8_t *lb = reinterpret_cast<const uint8_t *>(lds);
            uint32_t wv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const uint32_t p0 = st_pos[k][2 * q], p1 = st_pos[k][2 * q + 1];
              wv[q] = (uint32_t)lb[p0 & 0xffffu] | ((uint32_t)lb[p0 >> 16] << 8) |
                      ((uint32_t)lb[p1 & 0xffffu] << 16) | ((uint32_t)lb[p1 >> 16] << 24);
            }
            o.x = wv[0];
            o.y = wv[1];
            o.z = wv[2];
            o.w = wv[3];
          } else {
            o.x = lds[st_pos[k][0]];
            o.y = lds[st_pos[k][1]];
            o.z = lds[st_pos[k][2]];
            o.w = lds[st_pos[k][3]];
          }
          store16<NT>(dst + st_off[k] + cur * st_S[k], o);
        }
      __syncthreads();
    }
  }
}

__device__ inline uint64_t src_addr(const RArray &A, const RField &F, uint64_t r) {
  const RGroup &G = A.sgrp[F.sg];
  return G.base + (r >> G.logT) * ((uint64_t)G.S << G.logT) + ((uint64_t)F.sp << G.logT) +
         (r & ((1ull << G.logT) - 1)) * F.e;
}

__global__ __launch_bounds__(kBlock) void remap_tail_kernel(const RArray *__restrict__ arrays,
                                                            const RTail *__restrict__ regions,
                                                            uint32_t n_regions,
                                                            const uint8_t *src_override,
                                                            uint8_t *dst_override) {
  const uint64_t b = blockIdx.x;
  uint32_t lo = 0, hi = n_regions;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (regions[mid].block_begin <= b) lo = mid; else hi = mid;
  }
  const RTail Rg = regions[lo];
  const RArray &A = arrays[Rg.array];
  const RGroup &D = A.dgrp[Rg.dgroup];
  const uint8_t *src = src_override ? src_override : A.src;
  uint8_t *dst = dst_override ? dst_override : A.dst;
  const uint64_t first = Rg.start + (b - Rg.block_begin) * (uint64_t)kTailDwordsPerBlock * 4u;
  const uint64_t T = 1ull << D.logT, tileB = T * D.S;
  for (uint32_t i = threadIdx.x; i < kTailDwordsPerBlock; i += kBlock) {
    const uint64_t off = first + 4ull * i;
    if (off >= Rg.end) break;
    uint32_t word = 0;
    const uint64_t rel = off - D.base;
    if (rel < D.bytes && A.dword) {
      // 4- and 8-byte fields: the dword belongs to one field; decode it once
      const uint64_t w = rel >> 2, Sw = D.S >> 2;
      const uint64_t q = w / (T * Sw);
      const uint64_t within = w - q * T * Sw;
      const RField &F = A.fld[A.word_field[D.word_off + (uint32_t)(within >> D.logT)]];
      const uint64_t ew = F.e >> 2;
      const uint64_t local = within - ((uint64_t)(F.dp >> 2) << D.logT);
      const uint64_t rec = q * T + local / ew;
      const uint64_t jj = local % ew;
      if ((int64_t)rec < A.n) word = *reinterpret_cast<const uint32_t *>(src + src_addr(A, F, rec) + 4 * jj);
    } else if (rel < D.bytes) {
      for (uint32_t bi = 0; bi < 4; ++bi) {
        const uint64_t byte = rel + bi;
        const uint64_t q = byte / tileB;
        const uint64_t within = byte - q * tileB;
        const uint32_t col = (uint32_t)(within >> D.logT);
        const RField &F = A.fld[A.byte_field[D.byte_off + col]];
        const uint64_t local = within - ((uint64_t)F.dp << D.logT);
        const uint64_t rec = q * T + local / F.e;
        const uint64_t eb = local % F.e;
        if ((int64_t)rec < A.n) word |= (uint32_t)src[src_addr(A, F, rec) + eb] << (8 * bi);
      }
    }
    *reinterpret_cast<uint32_t *>(dst + off) = word;
  }
}

// ------------------------------------------------------------------ host side
static uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

uint32_t remap_lds_bytes(const LayoutDesc &a, const TileShape &s) {
  uint64_t D = (uint64_t)s.R * a.shape.record_bytes() / 4;
  if (D == 0) return 0;
  return (uint32_t)((D + ((D - 1) >> s.shift) + 1) * 4);
}

static constexpr uint32_t kMaxLds = 64 * 1024;

adha_status check_shape(const LayoutDesc &a, const LayoutDesc &b, const TileShape &s) {
  if (s.K != 1 && s.K != 2 && s.K != 4 && s.K != 8)
    return fail(ADHA_ERR_INVALID, "slots per thread must be 1, 2, 4 or 8 (got %u)", s.K);
  const uint32_t Tm = std::max(a.max_tile(), b.max_tile());
  const uint32_t Rmin = std::max<uint32_t>(64, Tm);
  if (s.R == 0 || s.R % Rmin)
    return fail(ADHA_ERR_INVALID, "tile of %u records is not a multiple of %u", s.R, Rmin);
  if (s.shift < 2 || s.shift > 31) return fail(ADHA_ERR_INVALID, "pad shift %u not in [2, 31]", s.shift);
  const uint64_t chunks = (uint64_t)s.R * a.shape.record_bytes() / 16;
  if (chunks > (uint64_t)kBlock * s.K)
    return fail(ADHA_ERR_INVALID, "tile of %u records needs %llu chunks > %u slots", s.R,
                (unsigned long long)chunks, kBlock * s.K);
  if (remap_lds_bytes(a, s) > kMaxLds) return fail(ADHA_ERR_INVALID, "tile needs more than 64 KiB of LDS");
  if (s.wg_per_cu == 0 || s.wg_per_cu > 32) return fail(ADHA_ERR_INVALID, "wg_per_cu not in [1, 32]");
  if (s.strided > 1 || s.nt > 1) return fail(ADHA_ERR_INVALID, "order and nontemporal flags are 0 or 1");
  return ADHA_OK;
}

adha_status policy_shape(const LayoutDesc &a, const LayoutDesc &b, uint32_t tile_bytes, uint32_t wg_per_cu,
                         uint32_t strided, uint32_t nt, TileShape *out) {
  TileShape s;
  s.shift = 6;
  s.wg_per_cu = wg_per_cu;
  s.strided = strided;
  s.nt = nt;
  const uint32_t S = a.shape.record_bytes();
  const uint32_t Rmin = std::max<uint32_t>(64, std::max(a.max_tile(), b.max_tile()));
  const uint64_t need = std::max<uint64_t>(tile_bytes, (uint64_t)Rmin * S);
  s.K = 1;
  while (s.K < 8 && (uint64_t)kBlock * 16 * s.K < need) s.K *= 2;
  if (S == 0 || (uint64_t)kBlock * 16 * s.K < (uint64_t)Rmin * S) {
    s.R = 0;
  } else {
    s.R = (uint32_t)(std::min<uint64_t>((uint64_t)kBlock * 16 * s.K, std::max<uint64_t>(tile_bytes, (uint64_t)Rmin * S)) /
                     S / Rmin * Rmin);
    if (remap_lds_bytes(a, s) > kMaxLds) s.R = 0;
  }
  *out = s;
  return ADHA_OK;
}

// Key of a layout pair's class for the tuning database: layout kinds, record
// bytes, largest tile, element-size class and log2 of the record count.
std::string tune_key(const LayoutDesc &a, const LayoutDesc &b) {
  uint32_t emask = 0;
  for (auto e : a.shape.ebytes) emask |= e;
  uint32_t lg = 0;
  while (lg < 62 && (int64_t(1) << (lg + 1)) <= a.shape.n) ++lg;
  char buf[160];
  snprintf(buf, sizeof buf, "pair:%d:%d:S%u:T%u:e%u:n%u", a.layout_class(), b.layout_class(),
           a.shape.record_bytes(), std::max(a.max_tile(), b.max_tile()), emask, lg);
  return buf;
}

// Default bytes per tile: 16 KiB in dword mode, the best measured for
// 64-byte records; 4 KiB in byte mode, whose sixteen positions per chunk
// make larger tiles cost occupancy (measured on 24-byte records of 1-, 2-
// and 4-byte fields: about 5.3 TB/s against 3.9 TB/s with 16 KiB tiles).
uint32_t default_tile_bytes(const LayoutDesc &a) { return a.dword_fields() ? 16384u : 4096u; }

// Default shape: a tuned entry for the pair's class if the context has one;
// otherwise default_tile_bytes per tile (at least max(64, T) records), 4
// workgroups per CU, strided tile order and streaming accesses.  R = 0 means
// "no full tiles": the tail kernel does everything (records too large for
// one tile).
adha_status choose_shape(const Ctx *ctx, const LayoutDesc &a, const LayoutDesc &b, TileShape *out) {
  if (ctx && !ctx->tunedb.empty()) {
    auto it = ctx->tunedb.find(tune_key(a, b));
    if (it != ctx->tunedb.end() && check_shape(a, b, it->second) >= 0) {
      *out = it->second;
      return ADHA_OK;
    }
  }
  return policy_shape(a, b, default_tile_bytes(a), 4, 1, 1, out);
}

// One device blob per launch: arrays, groups, fields, word tables, tails.
struct BlobBuilder {
  std::vector<uint8_t> bytes;
  // Appends n bytes copied from p (zeros when p is null); returns their offset.
  size_t add(const void *p, size_t n, size_t align = 16) {
    size_t at = (bytes.size() + align - 1) / align * align;
    bytes.resize(at + n, 0);
    if (p != nullptr && n != 0) memcpy(bytes.data() + at, p, n);
    return at;
  }
};

static void groups_of(const LayoutDesc &L, uint32_t R, std::vector<RGroup> &out,
                      std::vector<uint8_t> *words, std::vector<uint8_t> *bytes,
                      const std::vector<RField> *fl) {
  uint32_t tile_off = 0;
  for (size_t gi = 0; gi < L.groups.size(); ++gi) {
    const Group &g = L.groups[gi];
    RGroup r{};
    r.base = g.base;
    r.end = L.group_end(gi);
    r.bytes = g.bytes;
    r.S = g.S;
    r.logT = g.logT;
    r.tile_off = tile_off;
    tile_off += R * g.S;
    if (words) {
      r.word_off = (uint32_t)words->size();
      for (uint32_t w = 0; w < g.S / 4; ++w) {
        uint8_t fsel = 0;
        for (int f : g.fields)
          if ((*fl)[f].dp / 4 <= w && w < ((*fl)[f].dp + (*fl)[f].e) / 4) fsel = (uint8_t)f;
        words->push_back(fsel);
      }
    }
    if (bytes) {
      r.byte_off = (uint32_t)bytes->size();
      for (uint32_t b = 0; b < g.S; ++b) {
        uint8_t fsel = 0;
        for (int f : g.fields)
          if ((*fl)[f].dp <= b && b < (*fl)[f].dp + (*fl)[f].e) fsel = (uint8_t)f;
        bytes->push_back(fsel);
      }
    }
    out.push_back(r);
  }
}

adha_status remap_prepare(Ctx *ctx, const std::vector<const LayoutDesc *> &src_l,
                          const std::vector<const void *> &src,
                          const std::vector<const LayoutDesc *> &dst_l,
                          const std::vector<void *> &dst, const std::vector<TileShape> &shapes,
                          RemapPrepared *out, bool upload) {
  const size_t na = src_l.size();
  // Per array: groups, fields and word tables, collected first so that all
  // offsets are known; device pointers are patched in after allocation.
  struct Pending {
    RArray arr;
    size_t sg_at, dg_at, fl_at, wf_at, bf_at;
  };
  std::vector<Pending> pend(na);
  BlobBuilder blob;
  std::vector<RTail> tails;
  RemapPrepared P;
  std::vector<uint32_t> main_list;

  for (size_t i = 0; i < na; ++i) {
    const LayoutDesc &A = *src_l[i], &B = *dst_l[i];
    const TileShape &sh = shapes[i];
    const int F = A.shape.nfields();
    std::vector<RField> fl(F);
    for (int f = 0; f < F; ++f) {
      fl[f].sg = A.group_of[f];
      fl[f].dg = B.group_of[f];
      fl[f].sp = A.p[f];
      fl[f].dp = B.p[f];
      fl[f].e = A.shape.ebytes[f];
    }
    const uint32_t R = sh.R;
    std::vector<RGroup> sg, dg;
    std::vector<uint8_t> words, bytes;
    groups_of(A, R, sg, nullptr, nullptr, nullptr);
    groups_of(B, R, dg, B.dword_fields() ? &words : nullptr, &bytes, &fl);
    Pending &Q = pend[i];
    memset(&Q.arr, 0, sizeof Q.arr);
    Q.arr.n = A.shape.n;
    Q.arr.R = R;
    Q.arr.n_full = R ? (uint64_t)A.shape.n / R : 0;
    Q.arr.n_chunks = R ? (uint32_t)((uint64_t)R * A.shape.record_bytes() / 16) : 0;
    Q.arr.nsg = (uint32_t)sg.size();
    Q.arr.ndg = (uint32_t)dg.size();
    Q.arr.nf = (uint32_t)F;
    Q.arr.dword = B.dword_fields() ? 1u : 0u;
    Q.sg_at = blob.add(sg.data(), sg.size() * sizeof(RGroup));
    Q.dg_at = blob.add(dg.data(), dg.size() * sizeof(RGroup));
    Q.fl_at = blob.add(fl.data(), fl.size() * sizeof(RField));
    Q.wf_at = blob.add(words.data(), words.size(), 4);
    Q.bf_at = blob.add(bytes.data(), bytes.size(), 4);
    if (Q.arr.n_full > 0) {
      if (!Q.arr.dword) P.byte_path = 1;
      Q.arr.tile_begin = P.main_tiles;
      P.main_tiles += Q.arr.n_full;
      main_list.push_back((uint32_t)i);
      P.K = std::max(P.K, sh.K);
      P.shift = sh.shift;
      P.strided = sh.strided;
      P.nt = sh.nt;
      P.wg_per_cu = std::max(P.wg_per_cu, sh.wg_per_cu);
      P.lds = std::max(P.lds, remap_lds_bytes(A, sh));
    }
    // tail regions: everything in each destination group past the full tiles
    const uint64_t done = Q.arr.n_full * R;
    for (size_t gi = 0; gi < B.groups.size(); ++gi) {
      const uint64_t start = B.groups[gi].base + done * B.groups[gi].S;
      const uint64_t end = B.group_end(gi);
      if (end <= start) continue;
      RTail tr{};
      tr.array = (uint32_t)i;
      tr.dgroup = (uint32_t)gi;
      tr.start = start;
      tr.end = end;
      tr.block_begin = P.tail_blocks;
      P.tail_blocks += ceil_div(end - start, 4ull * kTailDwordsPerBlock);
      tails.push_back(tr);
    }
  }
  P.n_main = (uint32_t)main_list.size();
  P.n_tails = (uint32_t)tails.size();
  P.n_arrays = (uint32_t)na;
  if (P.main_tiles > 0) {
    const uint64_t want = (uint64_t)ctx->cu_count * P.wg_per_cu;
    uint64_t grid = std::min<uint64_t>(P.main_tiles, want);
    P.tiles_per_wg = ceil_div(P.main_tiles, grid);
    P.grid = ceil_div(P.main_tiles, P.tiles_per_wg);
  }

  const size_t arr_at = blob.add(nullptr, std::max<size_t>(1, na) * sizeof(RArray));
  const size_t main_at = blob.add(nullptr, std::max<size_t>(1, main_list.size()) * sizeof(RArray));
  const size_t tail_at = blob.add(tails.data(), tails.size() * sizeof(RTail));
  P.desc_bytes = blob.bytes.size();
  for (const RTail &tr : tails) P.tail_bytes += tr.end - tr.start;
  if (!upload) {  // host-side description only
    *out = P;
    return ADHA_OK;
  }

  uint8_t *dev = nullptr;
  hipError_t he = hipMalloc((void **)&dev, blob.bytes.size());
  if (he != hipSuccess) return fail(ADHA_ERR_OOM, "descriptor allocation failed: %s", hipGetErrorString(he));
  for (size_t i = 0; i < na; ++i) {
    Pending &Q = pend[i];
    Q.arr.src = (const uint8_t *)src[i];
    Q.arr.dst = (uint8_t *)dst[i];
    Q.arr.sgrp = (const RGroup *)(dev + Q.sg_at);
    Q.arr.dgrp = (const RGroup *)(dev + Q.dg_at);
    Q.arr.fld = (const RField *)(dev + Q.fl_at);
    Q.arr.word_field = dev + Q.wf_at;
    Q.arr.byte_field = dev + Q.bf_at;
    memcpy(blob.bytes.data() + arr_at + i * sizeof(RArray), &Q.arr, sizeof(RArray));
  }
  for (size_t j = 0; j < main_list.size(); ++j)
    memcpy(blob.bytes.data() + main_at + j * sizeof(RArray), &pend[main_list[j]].arr, sizeof(RArray));
  he = hipMemcpy(dev, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice);
  if (he != hipSuccess) {
    (void)hipFree(dev);
    return fail(ADHA_ERR_DEVICE, "descriptor upload failed: %s", hipGetErrorString(he));
  }
  P.dev = dev;
  P.arrays = dev + arr_at;
  P.main_arrays = dev + main_at;
  P.tails = dev + tail_at;
  *out = P;
  return ADHA_OK;
}

adha_status remap_run(Ctx *ctx, const RemapPrepared &P, const void *src_override,
                      void *dst_override, hipStream_t stream) {
  (void)ctx;
  const uint8_t *so = (const uint8_t *)src_override;
  uint8_t *dov = (uint8_t *)dst_override;
  if (P.main_tiles > 0) {
    const RArray *arrs = (const RArray *)P.main_arrays;
    const dim3 grid((uint32_t)P.grid), block(kBlock);
    const uint32_t sd = P.strided;
#define ADHA_REMAP_LAUNCH(KK, NTT, BYY)                                                             \
  hipLaunchKernelGGL((remap_tiles_kernel<KK, NTT, BYY>), grid, block, P.lds, stream, arrs, P.n_main, \
                     P.main_tiles, P.tiles_per_wg, P.shift, sd, so, dov)
#define ADHA_REMAP_K(NTT, BYY)                   \
  switch (P.K) {                                 \
    case 1: ADHA_REMAP_LAUNCH(1, NTT, BYY); break; \
    case 2: ADHA_REMAP_LAUNCH(2, NTT, BYY); break; \
    case 4: ADHA_REMAP_LAUNCH(4, NTT, BYY); break; \
    default: ADHA_REMAP_LAUNCH(8, NTT, BYY); break; \
  }
    if (P.byte_path) {
      if (P.nt) ADHA_REMAP_K(true, true) else ADHA_REMAP_K(false, true)
    } else {
      if (P.nt) ADHA_REMAP_K(true, false) else ADHA_REMAP_K(false, false)
    }
#undef ADHA_REMAP_K
#undef ADHA_REMAP_LAUNCH
    ADHA_HIP(hipGetLastError());
  }
  if (P.n_tails > 0) {
    hipLaunchKernelGGL(remap_tail_kernel, dim3((uint32_t)P.tail_blocks), dim3(kBlock), 0, stream,
                       (const RArray *)P.arrays, (const RTail *)P.tails, P.n_tails, so, dov);
    ADHA_HIP(hipGetLastError());
  }
  return ADHA_OK;
}

}  // namespace adha
